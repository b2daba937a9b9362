"""GPU parity at the benchmark sizes, in the configuration bench.py times
(float64 V(2,1), eta = 4, gamma = 2, graph replay, the default tile shapes).

The oracle finishes these sizes in seconds: assembly and hierarchy of the
flower at N = 4096 take about 8 s, a cycle about 0.4 s.  Compared:
  * every cell's type and lambda_K; the rows of A, M, G at every cut-cell
    vertex and at sampled interior rows; sampled rows of every Galerkin level;
  * the converged solution (1e-10 relative max difference), the cycle count
    and the per-cycle convergence factors (within 0.02), flower and ellipse;
  * mixed precision: error against the float64 oracle solution, of the size
    the residual tolerance allows;
  * the adjoint at N = 2048: lambda, dJ/df, dJ/dg after the transposed cycles,
    and central finite differences on 32 seeded directions;
  * problems of the 256-ellipse batched draw at their own sizes.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import assembly as oasm
from oracle import multigrid as omg

from helpers import rel_max

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_05105_amd as mg
    return mg


_cache = {}


def _oracle(name, N):
    key = (name, N)
    if key not in _cache:
        p = {"flower": W.flower_mms, "ellipse": W.ellipse_mms}[name](N)
        d = oasm.assemble(p.psi, N)
        H = omg.build_hierarchy(d)
        F = d.rhs(p.f, p.g)
        ref = omg.solve(H, F, tol=1e-10, max_cycles=60)
        _cache[key] = (p, d, H, F, ref)
    return _cache[key]


def _row_planes(A, rows, N):
    """The 9-point planes of the given CSR rows: out[p, r] = A[row, row + di + dj (N+1)]."""
    s = N + 1
    sub = A[rows].tocoo()
    out = np.zeros((9, len(rows)))
    k = np.asarray(rows)[sub.row]
    d = sub.col - k
    dj = np.rint(d / s).astype(int)
    di = d - dj * s
    assert np.all(np.abs(di) <= 1) and np.all(np.abs(dj) <= 1)
    np.add.at(out, ((di + 1) + 3 * (dj + 1), sub.row), sub.data)
    return out


def _gpu_planes(s, mg, what, level, rows):
    planes = s.export(what, level)
    n = planes.numel() // 9
    idx = torch.tensor(np.asarray(rows), device=planes.device, dtype=torch.int64)
    return planes.view(9, n)[:, idx].cpu().numpy()


def test_geometry_and_stencils_at_n4096():
    mg = _gpu()
    N = 4096
    p, d, H, F, ref = _oracle("flower", N)
    s = mg.Solver(p.psi, N)
    assert np.array_equal(s.export(mg._lib.EXPORT_PSI).cpu().numpy(), d.psi)
    assert s.info()["n_active"] == int(d.active.sum()) == 3370114
    ct = s.export(mg._lib.EXPORT_CELL_TYPE).cpu().numpy()
    assert np.array_equal(ct.astype(np.int64), d.cell_type.astype(np.int64))
    lam = s.export(mg._lib.EXPORT_CELL_LAMBDA).cpu().numpy()
    cut = d.cut_cells
    assert len(cut) > 9000
    assert rel_max(lam[cut], d.cell_lambda[cut]) < 1e-12
    # rows: every cut-cell vertex and 5000 sampled interior rows
    fl = s.export(mg._lib.EXPORT_NODE_FLAGS).cpu().numpy().astype(np.int64)
    stored = np.nonzero(fl & 2)[0]
    rng = np.random.default_rng(7)
    regular = rng.choice(np.nonzero((fl & 1) & ~(fl & 2))[0], 5000, replace=False)
    rows = np.concatenate([stored, regular])
    for what, M in ((mg._lib.EXPORT_A, d.A), (mg._lib.EXPORT_M, d.M), (mg._lib.EXPORT_G, d.G)):
        g = _gpu_planes(s, mg, what, 0, rows)
        o = _row_planes(M, rows, N)
        scale = np.abs(o).max()
        assert np.abs(g - o).max() <= 1e-12 * scale, what
    # Galerkin levels: sampled rows of every level against the oracle's R A P
    for lv in range(1, s.n_levels):
        Nl = s.level_n(lv)
        Al = H.levels[lv].A
        act = np.nonzero(np.abs(Al.diagonal()) > 0)[0]
        rows = act if len(act) <= 4000 else rng.choice(act, 4000, replace=False)
        g = _gpu_planes(s, mg, mg._lib.EXPORT_A, lv, rows)
        o = _row_planes(Al, rows, Nl)
        assert np.abs(g - o).max() <= 1e-11 * np.abs(o).max(), lv


@pytest.mark.parametrize("name,N", [("flower", 1024), ("flower", 2048), ("flower", 4096), ("ellipse", 4096)])
def test_converged_solution_at_benchmark_sizes(name, N):
    """The flower at N = 1024 and 2048 (float64 to 1e-10, extra smoothing on
    the cut cells) and both N = 4096 domains."""
    mg = _gpu()
    p, d, H, F, ref = _oracle(name, N)
    assert ref.converged
    s = mg.Solver(p.psi, N)
    u, hist = s.solve(p.f, p.g, tol=1e-10, max_cycles=60)
    assert s.last_status == 0
    assert len(hist) == len(ref.hist)
    ug = u.cpu().numpy()
    assert rel_max(ug, ref.u) < 1e-10
    assert np.abs(hist[1:] / hist[:-1] - ref.rho).max() < 0.02
    # each norm is of a residual F - A u whose rounding is of size
    # (stencil size) eps ||F||, whatever the residual's own size
    np.testing.assert_allclose(hist, ref.hist, rtol=1e-8, atol=50 * 2.2e-16 * hist[0])
    assert hist[-1] <= 1e-10 * np.abs(F).max()
    assert np.all(ug[~d.active] == 0)


@pytest.mark.parametrize("name", ["flower", "ellipse"])
def test_mixed_precision_error_at_n4096(name):
    """Float32 cycles inside float64 defect correction on both N = 4096
    domains, one or three float32 cycles per float64 step: the error against
    the float64 oracle solution (solved to 1e-14) is of the size the 1e-10
    residual tolerance allows, as for the float64 solve."""
    mg = _gpu()
    N = 4096
    p, d, H, F, ref = _oracle(name, N)
    tight = omg.solve(H, F, tol=1e-14, max_cycles=60, u0=ref.u)
    s64 = mg.Solver(p.psi, N)
    u64, _ = s64.solve(p.f, p.g, tol=1e-10)
    err64 = rel_max(u64.cpu().numpy(), tight.u)
    s64.close()
    for inner in (1, 3):
        s = mg.Solver(p.psi, N, precision=mg.PREC_MIXED, inner_cycles=inner)
        u, hist = s.solve(p.f, p.g, tol=1e-10)
        assert s.last_status == 0 and hist[-1] <= 1e-10 * np.abs(F).max()
        err = rel_max(u.cpu().numpy(), tight.u)
        print(f"{name} N={N}: mixed ({inner} float32 cycles per step) error vs float64 oracle {err:.3e} "
              f"(float64 solve {err64:.3e}), {len(hist) - 1} outer iterations")
        assert err < 10 * err64 + 1e-13, (inner, err, err64)
        s.close()


def test_adjoint_at_n2048():
    mg = _gpu()
    N = 2048
    p = W.flower_mms(N)
    d = oasm.assemble(p.psi, N)
    H = omg.build_hierarchy(d)
    ut = W.adjoint_target(N)
    k = 12
    s = mg.Solver(p.psi, N)
    u, _ = s.solve(p.f, p.g, tol=-1.0, max_cycles=k)
    J, dJdu = s.misfit(u, ut)
    uo = omg.solve(H, d.rhs(p.f, p.g), tol=-1.0, max_cycles=k).u
    Jo, dJduo = oadj.misfit(d, uo, ut)
    assert J == pytest.approx(Jo, rel=1e-11)
    df, dg, lam, _ = s.adjoint(dJdu, tol=-1.0, max_cycles=k)
    lamo = oadj.adjoint_solve(H, dJduo, tol=-1.0, max_cycles=k).u
    dfo, dgo = oadj.gradients(d, lamo)
    assert rel_max(lam.cpu().numpy(), lamo) < 1e-10
    assert rel_max(df.cpu().numpy(), dfo) < 1e-10
    assert rel_max(dg.cpu().numpy(), dgo) < 1e-10
    # central differences of J along 32 seeded directions, for f and for g
    f0 = torch.tensor(p.f, device="cuda:0")
    g0 = torch.tensor(p.g, device="cuda:0")
    utd = torch.tensor(ut, device="cuda:0")
    eps = 1e-6
    dirs = W.random_directions(d.n, 32, seed=1)

    def J_at(ff, gg):
        uu, _ = s.solve(ff, gg, tol=-1.0, max_cycles=k)
        return s.misfit(uu, utd)[0]

    for q, dv in enumerate(dirs):
        dvt = torch.tensor(dv, device="cuda:0")
        if q % 2 == 0:
            fd = (J_at(f0 + eps * dvt, g0) - J_at(f0 - eps * dvt, g0)) / (2 * eps)
            an = float(df @ dvt)
        else:
            fd = (J_at(f0, g0 + eps * dvt) - J_at(f0, g0 - eps * dvt)) / (2 * eps)
            an = float(dg @ dvt)
        # J is quadratic for a fixed cycle count: only rounding remains
        assert an == pytest.approx(fd, rel=1e-6, abs=50 * 2.2e-16 * abs(J) / eps), q


def test_batched_draw_sampled_problems():
    mg = _gpu()
    probs = W.batched_draws(count=256, seed=0)
    bs = mg.BatchedSolver([p.psi for p in probs], [p.N for p in probs])
    us, hists = bs.solve([p.f for p in probs], [p.g for p in probs], tol=1e-10, max_cycles=80)
    assert bs.last_status == 0
    for h in hists:
        assert h[-1] <= 1e-10 * h[0]
    # four problems of the largest size and a spread of the others
    pick = [i for i, p in enumerate(probs) if p.N == 512][:4] + list(range(0, 256, 37))
    for i in pick:
        p = probs[i]
        d = oasm.assemble(p.psi, p.N)
        F = d.rhs(p.f, p.g)
        ref = omg.solve(omg.build_hierarchy(d), F, tol=1e-14, max_cycles=100)
        ug = us[i].cpu().numpy()
        assert hists[i][0] == pytest.approx(np.abs(F).max(), rel=1e-12)
        assert np.all(ug[~d.active] == 0)
        s = mg.Solver(p.psi, p.N)
        u64, _ = s.solve(p.f, p.g, tol=1e-10, max_cycles=80)
        err64 = rel_max(u64.cpu().numpy(), ref.u)
        assert rel_max(ug, ref.u) < 10 * err64 + 1e-13, i
