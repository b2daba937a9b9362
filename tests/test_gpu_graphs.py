"""Graph replay of the solve loop against eager launches of the same kernels.

Each iteration of the solve loop is captured once and replayed; between
replays the host reads the residual norm and the caller's own stream work runs
(right-hand side, exports).  The replayed solves must equal the eager ones bit
for bit (same kernels, same order), on every solve of a sequence.
"""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_05105_amd as mg
    return mg


def _solver(mg, p, N, graphs, **kw):
    old = os.environ.get("MGFEM_NO_GRAPHS")
    os.environ["MGFEM_NO_GRAPHS"] = "0" if graphs else "1"
    try:
        return mg.Solver(p.psi, N, **kw)
    finally:
        if old is None:
            del os.environ["MGFEM_NO_GRAPHS"]
        else:
            os.environ["MGFEM_NO_GRAPHS"] = old


@pytest.mark.parametrize("kw", [{}, {"cycle": 2}, {"precision": 1}], ids=["V", "W", "mixed"])
def test_replayed_solves_equal_eager(kw):
    mg = _gpu()
    N = 256
    p = W.flower_mms(N)
    sg = _solver(mg, p, N, True, **kw)
    se = _solver(mg, p, N, False, **kw)
    rng = np.random.default_rng(5)
    for rep in range(3):
        f = p.f * (1.0 + 0.1 * rep) + 0.01 * rng.standard_normal(p.f.shape)
        ug, hg = sg.solve(f, p.g, tol=1e-10)
        ue, he = se.solve(f, p.g, tol=1e-10)
        torch.cuda.synchronize()
        assert len(hg) == len(he)
        assert np.array_equal(hg, he), (rep, hg, he)
        assert torch.equal(ug, ue), rep
        # the caller's own work between solves on the same stream
        ug.mul_(0.0)
    # a warm start and a fixed cycle count replay the same graphs
    ug, hg = sg.solve(p.f, p.g, tol=-1.0, max_cycles=4, u0=ue)
    ue2, he2 = se.solve(p.f, p.g, tol=-1.0, max_cycles=4, u0=ue)
    assert np.array_equal(hg, he2) and torch.equal(ug, ue2)


def test_replayed_adjoint_equals_eager():
    mg = _gpu()
    N = 256
    p = W.flower_mms(N)
    sg = _solver(mg, p, N, True)
    se = _solver(mg, p, N, False)
    u, _ = se.solve(p.f, p.g, tol=1e-10)
    J, dJdu = se.misfit(u, W.adjoint_target(N))
    for k in (3, 5, 3):
        a = sg.adjoint(dJdu, tol=-1.0, max_cycles=k)
        b = se.adjoint(dJdu, tol=-1.0, max_cycles=k)
        for x, y in zip(a[:3], b[:3]):
            assert torch.equal(x, y), k
        assert np.array_equal(a[3], b[3])


def test_profiled_replay_times_the_sweep():
    """Timing events inside the replayed graph: one timed launch per finest
    sweep, same results as the unprofiled solve."""
    mg = _gpu()
    N = 2048
    p = W.flower_mms(N)
    s = mg.Solver(p.psi, N)
    u0, h0 = s.solve(p.f, p.g, tol=1e-10)
    s.profile(True)
    u1, h1 = s.solve(p.f, p.g, tol=1e-10)
    prof = s.profile_read(0)
    s.profile(False)
    assert np.array_equal(h0, h1) and torch.equal(u0, u1)
    cycles = len(h1) - 1
    # three finest sweeps per cycle plus the speculative one of the last iteration
    assert prof["launches"] == 3 * cycles + 1
    assert prof["total_ms"] > 0 and prof["alg_bytes"] > 0
    # each timed launch repeated back to back: the same solve, one count per
    # launch, the alg. bytes of the matrix-free count (24 B per active row,
    # 72 B per stored row, 8 B per active coarse row with the prolongation)
    s.profile(True, repeat=5)
    u2, h2 = s.solve(p.f, p.g, tol=1e-10)
    prof5 = s.profile_read(0)
    s.profile(False)
    assert np.array_equal(h0, h2) and torch.equal(u0, u2)
    assert prof5["launches"] == prof["launches"]
    assert prof5["alg_bytes"] == prof["alg_bytes"]
    c0, c1 = s.level_counts(0), s.level_counts(1)
    expect = prof["launches"] * (24 * c0["n_active"] + 72 * c0["n_stored"]) + cycles * 8 * c1["n_active"]
    assert prof["alg_bytes"] == pytest.approx(expect, rel=1e-12)


def test_mixed_loop_queued_iteration_is_discarded():
    """The mixed loop queues its next iteration before reading the norm it
    waits for; when that norm meets the tolerance the queued iteration is
    dropped.  With every step at the full float32 cycle count, loose
    tolerances (the first cycles' factors improve on the factor the queueing
    predicts with) must return exactly the iterate and history of a run with
    the same number of cycles and no tolerance; with the last steps
    shortened from the residual history, the profiled loop (which never
    queues ahead) must agree bit for bit with the queueing one; and the
    solver must be unchanged for the next solve."""
    mg = _gpu()
    N = 256
    p = W.flower_mms(N)
    s = _solver(mg, p, N, True, precision=1)
    fresh = _solver(mg, p, N, True, precision=1)
    ref_u, ref_h = fresh.solve(p.f, p.g, tol=1e-10)
    for tol in (0.3, 0.1, 3e-2, 1e-3, 1e-6):
        os.environ["MGFEM_FIXED_INNER"] = "1"
        try:
            u, h = s.solve(p.f, p.g, tol=tol)
            assert list(s.step_cycles()) == [3] * (len(h) - 1)
            k = len(h) - 1
            assert s.last_status == 0 and h[-1] <= tol * h[0] < h[-2]  # u = 0: h[0] is the norm of F
            uf, hf = s.solve(p.f, p.g, tol=-1.0, max_cycles=k)
            torch.cuda.synchronize()
            assert np.array_equal(h, hf), tol
            assert torch.equal(u, uf), tol
        finally:
            del os.environ["MGFEM_FIXED_INNER"]
        u, h = s.solve(p.f, p.g, tol=tol)
        sc = s.step_cycles()
        assert s.last_status == 0 and h[-1] <= tol * h[0] and len(sc) == len(h) - 1
        s.profile(True)
        up, hp = s.solve(p.f, p.g, tol=tol)
        s.profile(False)
        assert np.array_equal(h, hp) and torch.equal(u, up), tol
        assert np.array_equal(sc, s.step_cycles()), tol
    u, h = s.solve(p.f, p.g, tol=1e-10)
    assert np.array_equal(h, ref_h) and torch.equal(u, ref_u)


def test_mixed_steps_shortened_from_the_history():
    """Step lengths: the full count while the target is far, fewer only for
    the last steps, never more in total than with every step at the full
    count, and the tolerance still met."""
    mg = _gpu()
    for name, N in (("flower", 1024), ("ellipse", 1024)):
        p = W.flower_mms(N) if name == "flower" else W.ellipse_mms(N)
        s = _solver(mg, p, N, True, precision=1)
        u, h = s.solve(p.f, p.g, tol=1e-10)
        sc = list(s.step_cycles())
        assert s.last_status == 0 and h[-1] <= 1e-10 * h[0] and len(sc) == len(h) - 1
        assert all(1 <= k <= 3 for k in sc) and sc[0] == 3
        # shortened steps come only at the end
        first_short = next((i for i, k in enumerate(sc) if k < 3), len(sc))
        assert len(sc) - first_short <= 2, sc
        os.environ["MGFEM_FIXED_INNER"] = "1"
        try:
            uf, hf = s.solve(p.f, p.g, tol=1e-10)
            scf = list(s.step_cycles())
        finally:
            del os.environ["MGFEM_FIXED_INNER"]
        assert scf == [3] * (len(hf) - 1)
        assert sum(sc) <= sum(scf), (name, sc, scf)
        print(f"{name} N={N}: float32 cycles per step {sc} (fixed: {scf})")
    # a float64 solve runs one cycle per iteration
    s64 = _solver(mg, p, N, True)
    u, h = s64.solve(p.f, p.g, tol=1e-10)
    assert list(s64.step_cycles()) == [1] * (len(h) - 1)


def test_list_smoother_without_group_plans():
    """MGFEM_NO_CUT_GROUPS=1 at set-up: the extra smoothing runs as one launch
    per colour over the cut-vertex list (the path of a level whose groups do
    not fit in LDS) instead of the grouped kernel.  Same cycles up to
    rounding (1/a_ii multiplied there, divided here), both against the oracle,
    eager and replayed, float64 and mixed."""
    mg = _gpu()
    from oracle import assembly as oasm
    from oracle import multigrid as omg
    N = 256
    p = W.flower_mms(N)
    d = oasm.assemble(p.psi, N)
    ref = omg.solve(omg.build_hierarchy(d), d.rhs(p.f, p.g), tol=-1.0, max_cycles=3)
    old = os.environ.get("MGFEM_NO_CUT_GROUPS")
    os.environ["MGFEM_NO_CUT_GROUPS"] = "1"
    try:
        sl = _solver(mg, p, N, True)
        sle = _solver(mg, p, N, False)
        slm = _solver(mg, p, N, True, precision=1, inner_cycles=1)
    finally:
        if old is None:
            del os.environ["MGFEM_NO_CUT_GROUPS"]
        else:
            os.environ["MGFEM_NO_CUT_GROUPS"] = old
    sg = _solver(mg, p, N, True)
    for s in (sl, sle, sg):
        u, h = s.solve(p.f, p.g, tol=-1.0, max_cycles=3)
        assert np.abs(u.cpu().numpy() - ref.u).max() <= 1e-10 * np.abs(ref.u).max()
    ul, hl = sl.solve(p.f, p.g, tol=1e-10)
    ug, hg = sg.solve(p.f, p.g, tol=1e-10)
    ule, hle = sle.solve(p.f, p.g, tol=1e-10)
    assert len(hl) == len(hg) and np.array_equal(hl, hle) and torch.equal(ul, ule)
    assert torch.abs(ul - ug).max() <= 1e-10 * torch.abs(ug).max()
    um, hm = slm.solve(p.f, p.g, tol=1e-10)
    assert slm.last_status == 0 and torch.abs(um - ug).max() <= 1e-8 * torch.abs(ug).max()


@pytest.mark.parametrize("inner", [1, 3])
def test_profiled_mixed_replay_times_the_float_sweep(inner):
    """Class 1: the float32 finest sweeps of the mixed cycles, three per
    float32 cycle and `inner` cycles per outer iteration; the profiled solve
    equals the unprofiled one."""
    mg = _gpu()
    N = 2048
    p = W.flower_mms(N)
    s = mg.Solver(p.psi, N, precision=mg.PREC_MIXED, inner_cycles=inner)
    u0, h0 = s.solve(p.f, p.g, tol=1e-10)
    s.profile(True)
    u1, h1 = s.solve(p.f, p.g, tol=1e-10)
    prof = s.profile_read(1)
    assert s.profile_read(0)["launches"] == 0
    s.profile(False)
    assert np.array_equal(h0, h1) and torch.equal(u0, u1)
    sc = s.step_cycles()
    assert len(sc) == len(h1) - 1 and all(1 <= k <= inner for k in sc)
    assert prof["launches"] == 3 * int(sc.sum())
    assert prof["total_ms"] > 0 and prof["alg_bytes"] > 0


def _solver_env(mg, p, N, env, **kw):
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return mg.Solver(p.psi, N, chi=p.chi, **kw)
    finally:
        for k, v in saved.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


@pytest.mark.parametrize("kw", [{}, {"cycle": 2}, {"cycle": 3}, {"precision": 1, "inner_cycles": 1}],
                         ids=["V", "W", "two_grid", "mixed"])
def test_coarse_map_equals_the_coarse_cycle(kw):
    """The coarse part applied as its precomputed dense map (the default)
    against the single-workgroup cycle it stands for (MGFEM_NO_COARSE_MAP=1):
    the same linear map, so iterates agree up to rounding, forward and
    transposed."""
    mg = _gpu()
    N = 256
    p = W.flower_mms(N)
    sm = _solver_env(mg, p, N, {"MGFEM_NO_COARSE_MAP": "0"}, **kw)
    sc = _solver_env(mg, p, N, {"MGFEM_NO_COARSE_MAP": "1"}, **kw)
    tol = 1e-5 if kw.get("precision") == 1 else 1e-12
    um, hm = sm.solve(p.f, p.g, tol=-1.0, max_cycles=4)
    uc, hc = sc.solve(p.f, p.g, tol=-1.0, max_cycles=4)
    scale = float(uc.abs().max())
    assert float((um - uc).abs().max()) <= tol * scale
    np.testing.assert_allclose(hm, hc, rtol=max(tol, 1e-9) * 100, atol=50 * 2.2e-16 * hc[0])
    if kw.get("precision") != 1:
        r = torch.tensor(np.random.default_rng(2).standard_normal(um.numel()), device=um.device)
        _, _, lm, _ = sm.adjoint(r, tol=-1.0, max_cycles=3)
        _, _, lc, _ = sc.adjoint(r, tol=-1.0, max_cycles=3)
        assert float((lm - lc).abs().max()) <= 1e-12 * float(lc.abs().max())
