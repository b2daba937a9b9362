#!/usr/bin/env python3
"""Benchmark: fine-grid DOF/s to 1e-10 relative residual at N = 4096.

Workload: the five-petal flower r - 0.5 - 0.1 sin(5 theta) about (0.02, 0.03)
on [-1, 1]^2 with N = 4096 cells per side (16.8M grid nodes), manufactured
solution u = sin(pi x) cos(pi y) + x^2, Q1 ghost FEM with lambda_K = 2 C(K),
V(2,1) cycles with four-colour Gauss-Seidel and 4 extra cut-cell sweeps,
stopping at ||F - A u||_inf <= 1e-10 ||F||_inf.

A step is one solve (right-hand side assembly, cycles and the per-cycle
residual norms) on inputs already resident in device memory; setup is timed
separately.  `value` is the FP64 form; the mixed-precision form (FP32 cycles in
FP64 defect correction) is reported beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine-grid DOF/s to 1e-10 rel. residual at N=4096 (FP64 vs mixed); HBM GB/s"
HBM_PEAK_GBS = 8000.0
SWEEP_KERNEL = "k_sweep<double, 64, 32, 512>"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic.json")


def source_hash():
    """Hash of the code of the profiled kernel's sources, comments and blank
    space left out (counters go stale when the code changes)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("smoother.hip", "mgfem_internal.h"):
        with open(os.path.join(ROOT, "paper_2505_05105_amd", "csrc", name)) as fh:
            text = fh.read()
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(domain="flower", N=4096):
    """HBM bytes per launch of the sweep kernel from the committed counter runs,
    or None when they were taken on other sources or another workload."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash():
        return None
    for rec in t.get("records", []):
        if rec.get("workload") == {"domain": domain, "N": N}:
            return rec.get("bytes_per_launch")
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=4096)
    ap.add_argument("--domain", default="flower", choices=["flower", "ellipse"])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-solves", type=int, default=3, help="oracle solves timed (median reported)")
    ap.add_argument("--no-cpu-scaling", action="store_true",
                    help="skip the oracle at N = 1024, 2048 and the all-threads solve")
    ap.add_argument("--profile-repeat", type=int, default=10,
                    help="each timed sweep launch repeated back to back between its events")
    ap.add_argument("--no-hbm", action="store_true", help="skip the N=16384 leg (working set above the MALL)")
    ap.add_argument("--hbm-N", type=int, default=16384)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--inner-cycles", type=int, default=3,
                    help="mixed precision (single and batched): float32 cycles per float64 defect-correction step")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched, adjoint and further-form legs")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the solves, run a plain 512 MiB device copy (counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(prob, N, solves):
    """The oracle, as it stands, on the same workload: its set-up (timed
    apart), then `solves` full solves to the same tolerance from zero; the
    median solve time gives DOF/s.  One thread (scipy's sparse products are
    single-threaded; BLAS pools are limited to one thread by the caller)."""
    import numpy as np
    from oracle import assembly as oasm
    from oracle import multigrid as omg
    t0 = time.perf_counter()
    d = oasm.assemble(prob.psi, N)
    H = omg.build_hierarchy(d)
    t1 = time.perf_counter()
    times, res = [], None
    for _ in range(solves):
        ts = time.perf_counter()
        F = d.rhs(prob.f, prob.g)
        res = omg.solve(H, F, tol=1e-10, max_cycles=60)
        times.append(time.perf_counter() - ts)
    med = float(np.median(times))
    dof = int(d.active.sum())
    return {
        "value": dof / med, "unit": "DOF/s", "cores": 1, "kind": "oracle",
        "sample": f"numpy/scipy oracle at N={N}: set-up ({t1 - t0:.1f} s, not in the value), then {solves} "
                  f"full solves to 1e-10 ({res.cycles} cycles each), median {med:.2f} s",
        "setup_s": t1 - t0, "solve_s": times, "cycles": int(res.cycles),
        "hist": [float(x) for x in res.hist], "u": res.u,
        "cpu": _cpu_name(), "nproc": os.cpu_count(),
    }


def cpu_scaling(W, solves):
    """The oracle at the smaller flower sizes (N = 1024, 2048) on one
    thread, and at N = 4096 with the thread pools unlimited (one solve):
    median solve times, set-up apart."""
    import numpy as np
    from oracle import assembly as oasm
    from oracle import multigrid as omg
    out = {"by_size": []}
    with _one_thread():
        for n in (1024, 2048):
            prob = W.flower_mms(n)
            d = oasm.assemble(prob.psi, n)
            H = omg.build_hierarchy(d)
            times = []
            for _ in range(solves):
                ts = time.perf_counter()
                res = omg.solve(H, d.rhs(prob.f, prob.g), tol=1e-10, max_cycles=60)
                times.append(time.perf_counter() - ts)
            med = float(np.median(times))
            dof = int(d.active.sum())
            out["by_size"].append({"N": n, "dof": dof, "cycles": int(res.cycles), "median_s": med,
                                   "dof_per_s": dof / med, "cores": 1})
    prob = W.flower_mms(4096)
    d = oasm.assemble(prob.psi, 4096)
    H = omg.build_hierarchy(d)
    ts = time.perf_counter()
    res = omg.solve(H, d.rhs(prob.f, prob.g), tol=1e-10, max_cycles=60)
    t = time.perf_counter() - ts
    out["all_threads_n4096"] = {"solve_s": t, "dof_per_s": int(d.active.sum()) / t, "cores": os.cpu_count(),
                                "note": "thread pools unlimited; scipy's sparse products stay single-threaded"}
    return out


def bench_batched(args, mg, W, torch, dev):
    """Batched form: `args.batch` seeded random ellipses, N drawn from
    {64, 128, 256, 512}, f ~ U[-1, 1], g = 0, float32 cycles with float64
    refinement (`args.inner_cycles` float32 cycles per refinement step), the
    path the autotuner picks, against the plain float64 single-problem solver
    run over the same problems one after another."""
    import numpy as np
    probs = W.batched_draws(count=args.batch, seed=0)
    psis = [torch.tensor(p.psi, device=dev) for p in probs]
    fs = [torch.tensor(p.f, device=dev) for p in probs]
    gs = [torch.tensor(p.g, device=dev) for p in probs]
    Ns = [p.N for p in probs]
    t0 = time.perf_counter()
    bs = mg.BatchedSolver(psis, Ns, inner_cycles=args.inner_cycles)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    outs = [torch.empty((n + 1) ** 2, dtype=torch.float64, device=dev) for n in Ns]
    for _ in range(args.warmup):
        bs.solve(fs, gs, tol=args.tol, max_cycles=100, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, hists = bs.solve(fs, gs, tol=args.tol, max_cycles=100, outs=outs)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    dof = bs_info_dof(bs, mg)
    cycles = [len(h) - 1 for h in hists]
    worst = max(float(h[-1] / h[0]) for h in hists)
    log(f"[bench] batched x{len(probs)}: {ms:.2f} ms/batch ({bs.last_ms():.2f} ms kernel), "
        f"{dof / (ms * 1e-3) / 1e9:.3f} GDOF/s, tile {bs.tile}")
    tile = bs.tile
    bs.close()
    del outs
    # the plain float64 form on the same problems, one solve after another
    solvers = [mg.Solver(p, n) for p, n in zip(psis, Ns)]
    u1 = [torch.empty((n + 1) ** 2, dtype=torch.float64, device=dev) for n in Ns]
    for s, f, g, u in zip(solvers, fs, gs, u1):
        s.solve(f, g, tol=args.tol, max_cycles=100, out=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, f, g, u in zip(solvers, fs, gs, u1):
        s.solve(f, g, tol=args.tol, max_cycles=100, out=u)
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3
    for s in solvers:
        s.close()
    log(f"[bench] sequential fp64 over the same batch: {ms_seq:.1f} ms")
    return {"value": dof / (ms * 1e-3), "unit": "DOF/s", "ms_per_step": ms, "problems": len(probs),
            "active_dof": dof, "N_counts": {str(n): Ns.count(n) for n in sorted(set(Ns))},
            "cycles_max": max(cycles), "cycles_mean": float(np.mean(cycles)),
            "worst_final_rel_residual": worst, "autotuned_tile": tile, "inner_cycles": args.inner_cycles, "setup_s": setup_s,
            "fp64_sequential_ms": ms_seq, "speedup_vs_fp64_sequential": ms_seq / ms,
            "dtype": "f32 cycles / f64 refinement"}


def bs_info_dof(bs, mg):
    import ctypes as C
    from paper_2505_05105_amd import _lib
    inf = _lib.Info()
    _lib.check(_lib.lib().mgfem_query(bs.handle, C.byref(inf)), bs.handle)
    return inf.n_active


def bench_adjoint(args, mg, W, torch, dev):
    """Adjoint workload: flower, N = 2048, misfit against u_t = cos(2 pi x) sin(pi y);
    the transposed cycles run as many cycles as the forward solve took."""
    N = 2048
    prob = W.flower_mms(N)
    s = mg.Solver(prob.psi, N)
    f = torch.tensor(prob.f, device=dev)
    g = torch.tensor(prob.g, device=dev)
    ut = torch.tensor(W.adjoint_target(N), device=dev)
    u, hist = s.solve(f, g, tol=args.tol, max_cycles=100)
    k = len(hist) - 1
    _, dJdu = s.misfit(u, ut)
    for _ in range(args.warmup):
        s.adjoint(dJdu, tol=-1.0, max_cycles=k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        df, dg, lam, ha = s.adjoint(dJdu, tol=-1.0, max_cycles=k)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    dof = s.info()["n_active"]
    log(f"[bench] adjoint N={N}: {ms:.2f} ms ({k} transposed cycles)")
    s.close()
    return {"value": dof / (ms * 1e-3), "unit": "DOF/s", "ms_per_step": ms, "N": N, "active_dof": dof,
            "cycles": k, "final_rel_residual": float(ha[-1] / ha[0]), "dtype": "f64"}


def bench_next(args, mg, W, torch, dev, N=4096, oracle_N=1024, with_oracle=True):
    """The further forms at N = 4096 (float64, tol as the main leg): the
    W-cycle, the two-grid scheme, re-discretised coarse operators, the annulus
    with a Neumann outer circle, and the global stabilisation parameter; each
    with the oracle's time per cycle of the same form beside it, measured on a
    bounded sample (N = 1024, two cycles after its set-up; skipped with the
    CPU baseline)."""
    import numpy as np
    from oracle import assembly as oasm
    from oracle import multigrid as omg
    from oracle import geometry as ogeo
    fl = W.flower_mms(N)
    an = W.annulus_mms(N)
    forms = [
        ("w_cycle", fl, {"cycle": mg.CYCLE_W}),
        ("two_grid", fl, {"cycle": mg.CYCLE_TWO_GRID}),
        ("rediscretised", fl, {"coarse_op": mg.COARSE_REDISCRETISED}),
        ("annulus_neumann", an, {}),
        ("global_stab", fl, {"stab_rule": mg.STAB_GLOBAL}),
    ]
    out = {}
    for name, prob, kw in forms:
        t0 = time.perf_counter()
        s = mg.Solver(prob.psi, N, chi=prob.chi, **kw)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        f = torch.tensor(prob.f, device=dev)
        g = torch.tensor(prob.g, device=dev)
        gN = None if prob.gN is None else torch.tensor(prob.gN, device=dev)
        u = torch.empty((N + 1) ** 2, dtype=torch.float64, device=dev)
        cap = 100
        s.solve(f, g, tol=args.tol, max_cycles=cap, out=u, gN=gN, raise_on_fail=False)
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for _ in range(reps):
            _, h = s.solve(f, g, tol=args.tol, max_cycles=cap, out=u, gN=gN, raise_on_fail=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        inf = s.info()
        h = np.asarray(h)
        cyc = len(h) - 1
        rec = {"ms_per_solve": ms, "cycles": cyc, "converged": bool(s.last_status == 0),
               "final_rel_residual": float(h[-1] / h[0]), "last_factor": float(h[-1] / h[-2]) if cyc else None,
               "ms_per_cycle": ms / max(cyc, 1), "active_dof": inf["n_active"],
               "value": inf["n_active"] / (ms * 1e-3) if s.last_status == 0 else None, "unit": "DOF/s",
               "setup_ms": inf["setup_ms"], "setup_wall_ms": setup_ms, "dtype": "f64"}
        if name == "global_stab":
            rec["global_C_times_h"] = inf["global_C"] * 2.0 / N
            rec["lanczos_steps"] = inf["global_iters"]
        s.close()
        out[name] = rec
        log(f"[bench] next {name}: {ms:.2f} ms, {cyc} cycles")
        if not with_oracle:
            continue
        # the oracle, the same form at N = oracle_N: set-up, then two cycles
        po = W.flower_mms(oracle_N) if prob is fl else W.annulus_mms(oracle_N)
        akw = {"chi": po.chi} if po.chi is not None else {}
        t0 = time.perf_counter()
        if name == "global_stab":
            d = oasm.assemble(po.psi, oracle_N, rule=ogeo.STAB_GLOBAL, **akw)
        else:
            d = oasm.assemble(po.psi, oracle_N, **akw)
        if name == "two_grid":
            H = omg.two_grid(d)
        elif name == "rediscretised":
            H = omg.build_hierarchy(d, rediscretise=(po.psi, dict(akw)))
        else:
            H = omg.build_hierarchy(d)
        t1 = time.perf_counter()
        F = d.rhs(po.f, po.g, po.gN)
        omg.solve(H, F, tol=-1.0, max_cycles=2, gamma_star=2 if name == "w_cycle" else 1)
        t2 = time.perf_counter()
        rec["oracle"] = {"N": oracle_N, "setup_s": t1 - t0, "per_cycle_s": (t2 - t1) / 2, "cores": 1,
                         "kind": "oracle", "sample": f"N={oracle_N}: set-up, then 2 cycles"}
        log(f"[bench] next {name}: oracle {(t2 - t1) / 2:.2f} s/cycle at N={oracle_N}")
    return out


def sweep_roofline(solver, solve, kernel_class, steps, repeat, traffic):
    """Roofline of the finest-level sweep (class 0 float64, class 1 the float32
    sweep of the mixed cycles), measured live: the solves again with HIP events
    on the solver's stream around every launch of that kernel, each launch
    issued `repeat` times back to back between its two events (the sweep
    reads one iterate buffer and writes the other, so a repeat recomputes the
    same values) so that the event pair's dispatch gap is spread over the
    repeats.  Algorithmic bytes per launch (matrix-free count): 3 values per
    active row (iterate read and written, right-hand side), 9 per stored row,
    1 per active coarse row when the prolongation is fused; the one flag byte
    per node the kernel also reads is reported apart."""
    solver.profile(True, repeat=repeat)
    solve()  # captures the profiled graphs
    torch_sync()
    solver.profile(True, repeat=repeat)  # reset the counters
    t0 = time.perf_counter()
    for _ in range(steps):
        solve()
    torch_sync()
    prof_ms = (time.perf_counter() - t0) * 1e3 / steps
    prof = solver.profile_read(kernel_class)
    solver.profile(False)
    launches = max(prof["launches"], 1)
    avg_ms = prof["total_ms"] / launches
    alg = prof["alg_bytes"] / launches
    achieved = alg / (avg_ms * 1e-3) / 1e9
    vb = 8 if kernel_class == 0 else 4
    kernel = SWEEP_KERNEL if kernel_class == 0 else SWEEP_KERNEL.replace("double", "float")
    log(f"[bench] {kernel}: {prof['launches']} launches, avg {avg_ms * 1e3:.2f} us "
        f"(x{repeat} back to back), {alg / 1e6:.1f} MB algorithmic -> {achieved:.0f} GB/s")
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "avg_launch_us": avg_ms * 1e3, "alg_bytes_per_launch": alg,
            "flag_bytes_per_launch": solver.level_counts(0)["n_active"],
            "byte_model": f"{3 * vb} B per active row + {9 * vb} B per stored row + {vb} B per active "
                          f"coarse row when the prolongation is fused (matrix-free interior rows)",
            "launches": prof["launches"], "repeat_per_event_pair": repeat,
            "profiled_ms_per_step": prof_ms}


def torch_sync():
    import torch
    torch.cuda.synchronize()


def bench_hbm(args, mg, W, torch, dev):
    """The same float64 solve on the flower at N = args.hbm_N (16384: 53.8M
    active DOF, 268M grid nodes): its level-0 vectors (about 0.5 GB each over
    the active box) are far larger than the 256 MB last-level cache, so the
    finest sweep's bytes come from HBM.  Inputs are generated on the device
    with the flower workload's formulas."""
    N = args.hbm_N
    log(f"[bench] hbm leg: setup N={N} flower")
    psi, f, g = W.flower_mms_device(N, dev)
    t0 = time.perf_counter()
    s = mg.Solver(psi, N)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    del psi
    u = torch.empty((N + 1) ** 2, dtype=torch.float64, device=dev)

    def run():
        return s.solve(f, g, tol=args.tol, max_cycles=100, out=u)[1]

    hist = run()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 3))
    t0 = time.perf_counter()
    for _ in range(steps):
        hist = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    dof = s.info()["n_active"]
    log(f"[bench] hbm leg N={N}: {ms:.2f} ms/solve, {len(hist) - 1} cycles, {dof / (ms * 1e-3) / 1e9:.3f} GDOF/s")
    roof = sweep_roofline(s, run, 0, steps, args.profile_repeat, measured_traffic("flower", N))
    roof.update({"workload": f"flower ghost-FEM Poisson, N={N}, V(2,1), eta=4, gamma=2, rel_tol={args.tol:g}",
                 "N": N, "active_dof": dof, "cycles": len(hist) - 1, "ms_per_solve": ms,
                 "dof_per_s": dof / (ms * 1e-3), "setup_s": setup_s,
                 "final_rel_residual": float(hist[-1] / hist[0])})
    s.close()
    # the mixed-precision solve of the same problem (float32 cycles, float64
    # outer step): at this size the bytes of the large levels dominate
    psi = W.flower_mms_device(N, dev)[0]
    sm = mg.Solver(psi, N, precision=mg.PREC_MIXED, inner_cycles=args.inner_cycles)
    del psi
    um = torch.empty_like(u)
    _, hm = sm.solve(f, g, tol=args.tol, max_cycles=100, out=um)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, hm = sm.solve(f, g, tol=args.tol, max_cycles=100, out=um)
    torch.cuda.synchronize()
    msm = (time.perf_counter() - t0) * 1e3 / steps
    roof["mixed"] = {"ms_per_solve": msm, "dof_per_s": dof / (msm * 1e-3), "cycles": len(hm) - 1,
                     "inner_cycles": args.inner_cycles, "step_cycles": [int(k) for k in sm.step_cycles()],
                     "speedup_vs_fp64": ms / msm, "final_rel_residual": float(hm[-1] / hm[0]),
                     "rel_err_vs_fp64_gpu": float((um - u).abs().max() / u.abs().max())}
    log(f"[bench] hbm leg N={N} mixed: {msm:.2f} ms/solve, {len(hm) - 1} cycles, {ms / msm:.2f}x the float64 solve")
    sm.close()
    del f, g, u, um
    torch.cuda.empty_cache()
    return roof


def bench_ellipse_mixed(args, mg, W, torch, dev, with_oracle):
    """The ellipse (0.7, 0.35) rotated 0.3 at N = 4096: float64 and mixed
    solves to the same tolerance; the errors of both against the converged
    discrete solution (the float64 solver run to 1e-15), the mixed solution's
    distance to the float64 GPU solution and, with the oracle, to the
    oracle's float64 solution at the same tolerance (one set-up and one solve
    on a host core)."""
    N = 4096
    prob = W.ellipse_mms(N)
    f = torch.tensor(prob.f, device=dev)
    g = torch.tensor(prob.g, device=dev)
    psi = torch.tensor(prob.psi, device=dev)
    rec = {}
    sols = {}
    for name, prec in (("fp64", mg.PREC_FP64), ("mixed", mg.PREC_MIXED)):
        kw = {"inner_cycles": args.inner_cycles} if prec == mg.PREC_MIXED else {}
        s = mg.Solver(psi, N, precision=prec, **kw)
        u = torch.empty((N + 1) ** 2, dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            _, h = s.solve(f, g, tol=args.tol, max_cycles=100, out=u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, h = s.solve(f, g, tol=args.tol, max_cycles=100, out=u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        dof = s.info()["n_active"]
        rec[name] = {"ms_per_step": ms, "value": dof / (ms * 1e-3), "unit": "DOF/s", "cycles": len(h) - 1,
                     "final_rel_residual": float(h[-1] / h[0])}
        if prec == mg.PREC_MIXED:
            rec[name]["step_cycles"] = [int(k) for k in s.step_cycles()]
        sols[name] = u
        if prec == mg.PREC_FP64:
            # the converged discrete solution the errors of both forms are measured against
            sols["converged"] = torch.empty_like(u)
            s.solve(f, g, tol=1e-15, max_cycles=80, out=sols["converged"], raise_on_fail=False)
        s.close()
        log(f"[bench] ellipse {name}: {ms:.3f} ms/solve, {len(h) - 1} cycles")
    rec["active_dof"] = dof
    rec["mixed"]["speedup_vs_fp64"] = rec["fp64"]["ms_per_step"] / rec["mixed"]["ms_per_step"]
    u64, umx = sols["fp64"], sols["mixed"]
    rec["mixed"]["rel_err_vs_fp64_gpu"] = float((umx - u64).abs().max() / u64.abs().max())
    uc = sols["converged"]
    for name, uu in (("fp64", u64), ("mixed", umx)):
        rec[name]["rel_err_vs_converged"] = float((uu - uc).abs().max() / uc.abs().max())
    if with_oracle:
        from oracle import assembly as oasm
        from oracle import multigrid as omg
        d = oasm.assemble(prob.psi, N)
        ref = omg.solve(omg.build_hierarchy(d), d.rhs(prob.f, prob.g), tol=args.tol, max_cycles=60)
        uo = torch.tensor(ref.u, device=dev)
        scale = uo.abs().max()
        rec["mixed"]["rel_err_vs_fp64_oracle"] = float((umx - uo).abs().max() / scale)
        rec["fp64"]["rel_err_vs_fp64_oracle"] = float((u64 - uo).abs().max() / scale)
        rec["oracle_cycles"] = int(ref.cycles)
        log(f"[bench] ellipse: mixed error vs the float64 oracle {rec['mixed']['rel_err_vs_fp64_oracle']:.2e}")
    return rec


def _final_l2(solver):
    """||F - A u||_2 / ||F||_2 after the solver's last solve (it recorded it)."""
    l2 = solver.residual_l2()
    return float(l2[-1] / l2[0]) if len(l2) else None


def _one_thread():
    """The oracle timings run on one core: BLAS/OpenMP pools limited to one
    thread (scipy's sparse products are single-threaded anyway)."""
    try:
        import numpy  # noqa: F401  (load the pools first: only loaded ones are limited)
        import scipy.linalg  # noqa: F401
        import scipy.sparse.linalg  # noqa: F401
        from threadpoolctl import threadpool_limits
        return threadpool_limits(limits=1)
    except ImportError:  # no pools to limit
        import contextlib
        return contextlib.nullcontext()


def _cpu_name():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (--gpus 1); the solver has no "
                                   "multi-GPU path"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2505_05105_amd as mg
    import workloads as W

    dev = torch.device("cuda:0")
    N = args.N
    if N > 8192 and args.domain == "flower":
        # large grids: the inputs are generated on the device (the oracle
        # baseline, which needs them on the host, is skipped at this size)
        prob = None
        psi, f, g = W.flower_mms_device(N, dev)
        args.no_cpu_baseline = True
    else:
        prob = W.flower_mms(N) if args.domain == "flower" else W.ellipse_mms(N)
        f = torch.tensor(prob.f, device=dev)
        g = torch.tensor(prob.g, device=dev)
        psi = torch.tensor(prob.psi, device=dev)
    log(f"[bench] setup N={N} {args.domain}")
    s64 = mg.Solver(psi, N)
    info = s64.info()
    dof = info["n_active"]
    u = torch.empty((N + 1) ** 2, dtype=torch.float64, device=dev)

    def run(solver, out):
        _, hist = solver.solve(f, g, tol=args.tol, max_cycles=100, out=out)
        return hist

    for _ in range(args.warmup):
        hist = run(s64, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        hist = run(s64, u)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    cycles = len(hist) - 1
    log(f"[bench] fp64: {ms:.3f} ms/solve, {cycles} cycles, {dof / (ms * 1e-3) / 1e9:.3f} GDOF/s")
    roof = sweep_roofline(s64, lambda: run(s64, u), 0, args.steps, args.profile_repeat,
                          measured_traffic(args.domain, N))
    out = {
        "metric": METRIC, "value": dof / (ms * 1e-3), "unit": "DOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.domain} ghost-FEM Poisson, N={N}, V(2,1), eta=4, gamma=2, "
                               f"rel_tol={args.tol:g}", "N": N, "active_dof": dof,
                   "grid_nodes": (N + 1) ** 2, "cycles": cycles, "precision": "fp64"},
        "grid_nodes_per_s": (N + 1) ** 2 / (ms * 1e-3),
        "setup_ms": info["setup_ms"],
        "final_rel_residual": float(hist[-1] / hist[0]),
        "final_rel_residual_l2": _final_l2(s64),
        "roofline": roof,
        "levels": [dict(N=s64.level_n(l), **s64.level_counts(l)) for l in range(info["n_levels"])],
    }

    # the converged discrete solution (the same float64 solver run far past the
    # tolerance): what the errors of both forms at the 1e-10 residual are
    # measured against, beside their distance to the oracle at that tolerance
    ut = torch.empty_like(u)
    _, ht = s64.solve(f, g, tol=1e-15, max_cycles=80, out=ut, raise_on_fail=False)
    uts = float(ut.abs().max())
    out["fp64_rel_err_vs_converged"] = float((u - ut).abs().max()) / uts
    out["converged_reference"] = {"cycles": len(ht) - 1, "final_rel_residual": float(ht[-1] / ht[0])}

    u_mixed = None
    if not args.no_mixed:
        smx = mg.Solver(psi, N, precision=mg.PREC_MIXED, inner_cycles=args.inner_cycles)
        um = torch.empty_like(u)
        for _ in range(args.warmup):
            hm = run(smx, um)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            hm = run(smx, um)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        msm = (t1 - t0) * 1e3 / args.steps
        step_cycles = [int(k) for k in smx.step_cycles()]
        err = float((um - u).abs().max() / u.abs().max())
        u_mixed = um.cpu().numpy()
        # the float32 finest sweep timed the same way
        roof32 = sweep_roofline(smx, lambda: run(smx, um), 1, args.steps, args.profile_repeat, None)
        out["mixed"] = {"value": dof / (msm * 1e-3), "unit": "DOF/s", "ms_per_step": msm,
                        "cycles": len(hm) - 1, "inner_cycles": args.inner_cycles,
                        "float_cycles": sum(step_cycles), "step_cycles": step_cycles,
                        "dtype": "f32 cycles / f64 outer",
                        "rel_err_vs_fp64_gpu": err, "final_rel_residual": float(hm[-1] / hm[0]),
                        "speedup_vs_fp64": ms / msm, "roofline": roof32,
                        "rel_err_vs_converged": float((um - ut).abs().max()) / uts}
        log(f"[bench] mixed: {msm:.3f} ms/solve, {len(hm) - 1} cycles, err vs fp64 {err:.2e}")
        smx.close()

    u_fp64 = u.cpu().numpy()
    s64.close()
    if not args.no_hbm:
        del f, g, psi, u, ut
        torch.cuda.empty_cache()
        out["roofline_hbm"] = bench_hbm(args, mg, W, torch, dev)

    if not args.no_extras:
        with _one_thread():
            out["ellipse"] = bench_ellipse_mixed(args, mg, W, torch, dev, not args.no_cpu_baseline)
        out["batched"] = bench_batched(args, mg, W, torch, dev)
        out["adjoint"] = bench_adjoint(args, mg, W, torch, dev)
        with _one_thread():
            out["next"] = bench_next(args, mg, W, torch, dev, with_oracle=not args.no_cpu_baseline)

    if args.copy_probe:
        # a plain copy of known size: what FETCH_SIZE / WRITE_SIZE read for it calibrates the counters
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        torch.neg(a, out=b)  # one elementwise kernel: reads 512 MiB, writes 512 MiB
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = a.numel() * 8
        del a, b

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        with _one_thread():
            out["cpu_baseline"] = cpu_baseline(prob, N, args.cpu_solves)
        uo = out["cpu_baseline"].pop("u")
        if "mixed" in out and u_mixed is not None:
            out["mixed"]["rel_err_vs_fp64_oracle"] = float(np.abs(u_mixed - uo).max() / np.abs(uo).max())
        out["fp64_rel_err_vs_oracle"] = float(np.abs(u_fp64 - uo).max() / np.abs(uo).max())
        hc = np.array(out["cpu_baseline"].pop("hist"))
        out["cpu_baseline"]["same_cycle_count_as_gpu"] = len(hc) == len(hist)
        k = min(len(hc), len(hist))
        out["cpu_baseline"]["hist_rel_diff_vs_gpu"] = float(
            np.max(np.abs(hc[:k] - hist[:k]) / np.abs(hist[:k])))
        if args.domain == "flower" and N == 4096 and not args.no_cpu_scaling:
            log("[bench] cpu baseline at N = 1024, 2048 and on every thread")
            out["cpu_baseline"].update(cpu_scaling(W, args.cpu_solves))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
