"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Floating-point tolerances: setup quantities (lambda_K, stencils, Galerkin
operators) differ only by summation order and quadrature rule, so they agree
to ~1e-13 relative; iterates agree to rounding at equal cycle counts; converged
FP64 solutions within 1e-10 relative max difference and per-cycle convergence
factors within 0.02.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import assembly as oasm
from oracle import multigrid as omg

from helpers import planes_from_csr, rel_max

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_05105_amd as mg
    return mg


def _case(name, N):
    if name == "circle":
        p = W.circle_mms(N)
    elif name == "flower":
        p = W.flower_mms(N)
    elif name == "ellipse":
        p = W.ellipse_mms(N)
    elif name == "paper_flower":
        u, f = W.mms_flower(N)
        p = W.Problem("pf", N, W.paper_flower(N), f, u.copy(), u)
    else:
        raise ValueError(name)
    return p


_cache = {}


def oracle_for(name, N, **kw):
    key = (name, N, tuple(sorted(kw.items())))
    if key not in _cache:
        p = _case(name, N)
        d = oasm.assemble(p.psi, N, **kw)
        H = omg.build_hierarchy(d)
        _cache[key] = (p, d, H)
    return _cache[key]


CASES = [("circle", 64), ("flower", 128), ("ellipse", 64), ("paper_flower", 32)]


@pytest.mark.parametrize("name,N", CASES)
def test_geometry_and_stabilisation(name, N):
    mg = _gpu()
    p, d, _ = oracle_for(name, N)
    s = mg.Solver(p.psi, N)
    psi = s.export(mg._lib.EXPORT_PSI).cpu().numpy()
    assert np.array_equal(psi, d.psi)
    ct = s.export(mg._lib.EXPORT_CELL_TYPE).cpu().numpy().astype(int)
    assert np.array_equal(ct, d.cell_type)
    lam = s.export(mg._lib.EXPORT_CELL_LAMBDA).cpu().numpy()
    cut = d.cut_cells
    np.testing.assert_allclose(lam[cut], d.cell_lambda[cut], rtol=1e-12)
    assert np.all(lam[np.setdiff1d(np.arange(N * N), cut)] == 0)
    info = s.info()
    assert info["n_active"] == int(d.active.sum())
    counts = np.bincount(d.cell_type, minlength=7)
    assert list(info["n_cells_by_type"].values()) == counts.tolist()


@pytest.mark.parametrize("name,N", CASES)
def test_fine_stencils(name, N):
    mg = _gpu()
    p, d, _ = oracle_for(name, N)
    s = mg.Solver(p.psi, N)
    for what, mat in ((mg._lib.EXPORT_A, d.A), (mg._lib.EXPORT_M, d.M), (mg._lib.EXPORT_G, d.G)):
        got = s.export(what).cpu().numpy().reshape(9, -1)
        ref = planes_from_csr(mat, N)
        assert rel_max(got, ref) < 1e-13, what
    fl = s.export(mg._lib.EXPORT_NODE_FLAGS).cpu().numpy().astype(int)
    assert np.array_equal((fl & 1) == 1, d.active)


@pytest.mark.parametrize("name,N", CASES)
def test_galerkin_hierarchy(name, N):
    mg = _gpu()
    p, d, H = oracle_for(name, N)
    s = mg.Solver(p.psi, N)
    assert s.n_levels == len(H.levels)
    for l, lv in enumerate(H.levels):
        got = s.export(mg._lib.EXPORT_A, l).cpu().numpy().reshape(9, -1)
        ref = planes_from_csr(lv.A, lv.N)
        assert rel_max(got, ref) < 1e-12, l
        fl = s.export(mg._lib.EXPORT_NODE_FLAGS, l).cpu().numpy().astype(int)
        assert np.array_equal((fl & 1) == 1, lv.active), l
        if lv.cut is not None:
            assert np.array_equal((fl & 4) == 4, lv.cut), l


@pytest.mark.parametrize("level", [0, 1, 2])
@pytest.mark.parametrize("reverse", [False, True])
def test_single_smoothing_step(level, reverse):
    mg = _gpu()
    p, d, H = oracle_for("flower", 128)
    s = mg.Solver(p.psi, 128)
    lv = H.levels[level]
    rng = np.random.default_rng(level)
    x0 = rng.standard_normal(lv.A.shape[0]) * lv.active
    b = rng.standard_normal(lv.A.shape[0]) * lv.active
    xo = x0.copy()
    omg.smoothing_step(lv, xo, b, 4, reverse=reverse)
    xg = torch.tensor(x0, device="cuda:0")
    s.smooth(level, xg, torch.tensor(b, device="cuda:0"), 1, reverse)
    assert rel_max(xg.cpu().numpy(), xo) < 1e-13


@pytest.mark.parametrize("cycles", [1, 3])
def test_fixed_cycles_iterates(cycles):
    mg = _gpu()
    p, d, H = oracle_for("flower", 128)
    s = mg.Solver(p.psi, 128)
    u, hist = s.solve(p.f, p.g, tol=-1.0, max_cycles=cycles)
    ref = omg.solve(H, d.rhs(p.f, p.g), tol=-1.0, max_cycles=cycles)
    assert len(hist) == cycles + 1
    assert rel_max(u.cpu().numpy(), ref.u) < 1e-12
    np.testing.assert_allclose(hist, ref.hist, rtol=1e-9)
    F = s.export(mg._lib.EXPORT_RHS).cpu().numpy()
    assert rel_max(F, d.rhs(p.f, p.g)) < 1e-13


@pytest.mark.parametrize("name,N", [("circle", 64), ("flower", 256), ("ellipse", 128)])
def test_converged_solution_and_rho(name, N):
    mg = _gpu()
    p, d, H = oracle_for(name, N)
    s = mg.Solver(p.psi, N)
    u, hist = s.solve(p.f, p.g, tol=1e-10, max_cycles=60)
    ref = omg.solve(H, d.rhs(p.f, p.g), tol=1e-10, max_cycles=60)
    assert s.last_status == 0 and ref.converged
    assert len(hist) == len(ref.hist)
    assert rel_max(u.cpu().numpy(), ref.u) < 1e-10
    rho_g = hist[1:] / hist[:-1]
    assert np.abs(rho_g - ref.rho).max() < 0.02
    assert hist[-1] <= 1e-10 * np.abs(d.rhs(p.f, p.g)).max()
    # inactive nodes are zero
    assert np.all(u.cpu().numpy()[~d.active] == 0)


def test_w_cycle_parity():
    mg = _gpu()
    p, d, H = oracle_for("flower", 128)
    s = mg.Solver(p.psi, 128, cycle=mg.CYCLE_W)
    u, hist = s.solve(p.f, p.g, tol=-1.0, max_cycles=3)
    ref = omg.solve(H, d.rhs(p.f, p.g), tol=-1.0, max_cycles=3, gamma_star=2)
    assert rel_max(u.cpu().numpy(), ref.u) < 1e-12


def test_warm_start_continues():
    mg = _gpu()
    p, d, H = oracle_for("circle", 64)
    s = mg.Solver(p.psi, 64)
    u1, _ = s.solve(p.f, p.g, tol=-1.0, max_cycles=2)
    u2, _ = s.solve(p.f, p.g, tol=-1.0, max_cycles=1, u0=u1)
    ref = omg.solve(H, d.rhs(p.f, p.g), tol=-1.0, max_cycles=3)
    assert rel_max(u2.cpu().numpy(), ref.u) < 1e-12


@pytest.mark.parametrize("N", [256, 1024])
def test_mixed_outer_residual_matches_host_recomputation(N):
    """The float64 outer step of the mixed solve (over the level's sweep
    tiles: 16 x 16 at N = 256, 64 x 16 at N = 1024) reports the norms of
    F - A u for the iterate it returns: recomputed on the host from the
    library's own stencil planes (the oracle's agree with them only to
    ~1e-13, more than a small residual can tell apart) and the oracle's
    right-hand side after one and two steps, the max and l2 norms agree to
    the rounding of A u."""
    mg = _gpu()
    p, d, H = oracle_for("flower", N)
    F = d.rhs(p.f, p.g)
    s = mg.Solver(p.psi, N, precision=mg.PREC_MIXED)
    A = s.export(mg._lib.EXPORT_A, 0).cpu().numpy().reshape(9, N + 1, N + 1)
    for k in (1, 2):
        u, hist = s.solve(p.f, p.g, tol=-1.0, max_cycles=k)
        U = np.pad(u.cpu().numpy().reshape(N + 1, N + 1), 1)
        Au = np.zeros((N + 1, N + 1))
        for q in range(9):
            di, dj = q % 3 - 1, q // 3 - 1
            Au += A[q] * U[1 + dj:N + 2 + dj, 1 + di:N + 2 + di]
        r = (F - Au.reshape(-1)) * d.active
        floor = 64 * 2.2e-16 * 6 * np.abs(u.cpu().numpy()).max()
        assert hist[-1] > 1e3 * floor
        assert abs(np.abs(r).max() - hist[-1]) <= 1e-6 * hist[-1] + floor
        l2 = s.residual_l2()[-1]
        assert abs(np.linalg.norm(r) - l2) <= 1e-6 * l2 + floor * np.sqrt(d.n)


def test_mixed_precision_reaches_fp64_tolerance():
    """FP32 cycles inside FP64 defect correction reach the FP64 residual
    tolerance; the solution error against the FP64 oracle is then of the size
    the residual allows, the same as for the FP64 solve at that tolerance."""
    mg = _gpu()
    p, d, H = oracle_for("flower", 256)
    F = d.rhs(p.f, p.g)
    ref = omg.solve(H, F, tol=1e-14, max_cycles=80)
    s64 = mg.Solver(p.psi, 256)
    for inner in (1, 2, 3):
        s = mg.Solver(p.psi, 256, precision=mg.PREC_MIXED, inner_cycles=inner)
        for tol in (1e-10, 1e-12):
            u64, _ = s64.solve(p.f, p.g, tol=tol, max_cycles=80)
            err64 = rel_max(u64.cpu().numpy(), ref.u)
            u, hist = s.solve(p.f, p.g, tol=tol, max_cycles=80)
            assert s.last_status == 0
            assert hist[-1] <= tol * np.abs(F).max()
            err = rel_max(u.cpu().numpy(), ref.u)
            # the error is set by the residual tolerance, as for the FP64 solve
            assert err < 10 * err64 + 1e-13, (inner, tol, err, err64)
    with pytest.raises(mg.MgfemError):
        mg.Solver(p.psi, 256, precision=mg.PREC_MIXED, inner_cycles=0)


@pytest.mark.parametrize("k", [2, 5])
def test_adjoint_matches_oracle(k):
    mg = _gpu()
    p, d, H = oracle_for("flower", 128)
    s = mg.Solver(p.psi, 128)
    ut = W.adjoint_target(128)
    u, _ = s.solve(p.f, p.g, tol=-1.0, max_cycles=k)
    J, dJdu = s.misfit(u, ut)
    uo = omg.solve(H, d.rhs(p.f, p.g), tol=-1.0, max_cycles=k).u
    Jo, dJduo = oadj.misfit(d, uo, ut)
    assert J == pytest.approx(Jo, rel=1e-11)
    assert rel_max(dJdu.cpu().numpy(), dJduo) < 1e-11
    df, dg, lam, _ = s.adjoint(dJdu, tol=-1.0, max_cycles=k)
    lamo = oadj.adjoint_solve(H, dJduo, tol=-1.0, max_cycles=k).u
    dfo, dgo = oadj.gradients(d, lamo)
    assert rel_max(lam.cpu().numpy(), lamo) < 1e-11
    assert rel_max(df.cpu().numpy(), dfo) < 1e-11
    assert rel_max(dg.cpu().numpy(), dgo) < 1e-11


def test_autograd_function_matches_finite_differences():
    mg = _gpu()
    N = 64
    p, d, H = oracle_for("flower", N)
    s = mg.Solver(p.psi, N)
    ut = torch.tensor(W.adjoint_target(N), device="cuda:0")
    M = torch.tensor(planes_from_csr(d.M, N), device="cuda:0")
    f = torch.tensor(p.f, device="cuda:0", requires_grad=True)
    g = torch.tensor(p.g, device="cuda:0", requires_grad=True)
    k = 6

    def J_of(ff, gg):
        u = mg.GhostFEMSolve.apply(ff, gg, s, -1.0, k)
        J, _ = s.misfit(u.detach(), ut)
        return u, J

    u = mg.GhostFEMSolve.apply(f, g, s, -1.0, k)
    _, dJdu = s.misfit(u.detach(), ut)
    (u * dJdu).sum().backward()
    dirs = W.random_directions(d.n, 4, seed=1)
    eps = 1e-6
    for dv in dirs:
        dvt = torch.tensor(dv, device="cuda:0")
        for which, grad in (("f", f.grad), ("g", g.grad)):
            if which == "f":
                Jp = J_of(f.detach() + eps * dvt, g.detach())[1]
                Jm = J_of(f.detach() - eps * dvt, g.detach())[1]
            else:
                Jp = J_of(f.detach(), g.detach() + eps * dvt)[1]
                Jm = J_of(f.detach(), g.detach() - eps * dvt)[1]
            fd = (Jp - Jm) / (2 * eps)
            # J is quadratic in (f, g) for a fixed cycle count, so central
            # differences have no truncation error; what remains is rounding,
            # of size eps_mach |J| / eps
            J0 = J_of(f.detach(), g.detach())[1]
            assert float(grad @ dvt) == pytest.approx(fd, rel=1e-6, abs=50 * 2.2e-16 * abs(J0) / eps)
    del M
    # the backward pass is the transposed float64 cycle map: a mixed-precision
    # forward would not be its transpose, so such a solver is refused
    sm = mg.Solver(p.psi, N, precision=mg.PREC_MIXED)
    with pytest.raises(ValueError):
        mg.GhostFEMSolve.apply(f, g, sm, -1.0, k)


def test_stabilisation_rules():
    mg = _gpu()
    N = 64
    p = W.flower_mms(N)
    for rule, kw in ((mg.STAB_LOCAL_EIG, {}), (mg.STAB_FIXED, {"lambda_fixed": 300.0})):
        d = oasm.assemble(p.psi, N, rule=rule, **kw)
        s = mg.Solver(p.psi, N, stab_rule=rule, **kw)
        lam = s.export(mg._lib.EXPORT_CELL_LAMBDA).cpu().numpy()
        np.testing.assert_allclose(lam[d.cut_cells], d.cell_lambda[d.cut_cells], rtol=1e-9)
        got = s.export(mg._lib.EXPORT_A).cpu().numpy().reshape(9, -1)
        assert rel_max(got, planes_from_csr(d.A, N)) < 1e-10


def test_random_level_sets_with_saddles_and_box_contact():
    """Ragged inputs: noisy level sets produce saddle cells and touch the box."""
    mg = _gpu()
    N = 32
    rng = np.random.default_rng(7)
    seen_saddle = False
    for trial in range(6):
        psi = W.circle(N, radius=0.6 + 0.5 * (trial % 2)) + 0.05 * rng.standard_normal((N + 1) ** 2)
        d = oasm.assemble(psi, N)
        H = omg.build_hierarchy(d)
        seen_saddle |= bool(np.isin(d.cell_type, [5, 6]).any())
        s = mg.Solver(psi, N)
        ct = s.export(mg._lib.EXPORT_CELL_TYPE).cpu().numpy().astype(int)
        assert np.array_equal(ct, d.cell_type)
        got = s.export(mg._lib.EXPORT_A).cpu().numpy().reshape(9, -1)
        assert rel_max(got, planes_from_csr(d.A, N)) < 1e-12
        f = rng.uniform(-1, 1, d.n)
        g = rng.uniform(-1, 1, d.n)
        u, _ = s.solve(f, g, tol=-1.0, max_cycles=2)
        ref = omg.solve(H, d.rhs(f, g), tol=-1.0, max_cycles=2)
        assert rel_max(u.cpu().numpy(), ref.u) < 1e-11
    assert seen_saddle


def test_error_paths():
    mg = _gpu()
    N = 32
    with pytest.raises(mg.MgfemError) as e:
        mg.Solver(np.ones((N + 1) ** 2), N)  # nothing inside
    assert e.value.code == mg._lib.ERR_EMPTY_DOMAIN
    with pytest.raises(mg.MgfemError):
        mg.Solver(W.circle(N), N, gamma=0.5)
    p = W.circle_mms(N)
    s = mg.Solver(p.psi, N)
    u, hist = s.solve(p.f, p.g, tol=1e-14, max_cycles=1, raise_on_fail=False)
    assert s.last_status == mg._lib.ERR_NOT_CONVERGED and len(hist) == 2
    # a fixed lambda far below C(K) loses coercivity (section 4.4): either the
    # coarsest factorisation fails or the cycles do not converge
    try:
        bad = mg.Solver(p.psi, N, stab_rule=mg.STAB_FIXED, lambda_fixed=1e-3)
    except mg.MgfemError as err:
        assert err.code == mg._lib.ERR_SINGULAR_COARSE
    else:
        u, hist = bad.solve(p.f, p.g, tol=1e-10, max_cycles=40, raise_on_fail=False)
        assert bad.last_status in (mg._lib.ERR_DIVERGED, mg._lib.ERR_NOT_CONVERGED)


def test_residual_l2_history_matches_oracle():
    """The l2 residual norms beside the max-norm history (section 3.1 uses
    the max norm; both are recorded), float64 forward, adjoint and mixed."""
    mg = _gpu()
    N = 128
    p = W.flower_mms(N)
    d = oasm.assemble(p.psi, N)
    H = omg.build_hierarchy(d)
    F = d.rhs(p.f, p.g)
    s = mg.Solver(p.psi, N)
    u, hist = s.solve(p.f, p.g, tol=1e-10)
    ref = omg.solve(H, F, tol=1e-10)
    l2 = s.residual_l2()
    assert len(l2) == len(hist) == len(ref.hist_l2)
    np.testing.assert_allclose(l2, ref.hist_l2, rtol=1e-8, atol=50 * 2.2e-16 * ref.hist_l2[0])
    r = np.random.default_rng(2).standard_normal(d.n) * d.active
    _, _, lam, ah = s.adjoint(r, tol=-1.0, max_cycles=3)
    from oracle import adjoint as oadj
    aref = oadj.adjoint_solve(H, r, tol=-1.0, max_cycles=3)
    np.testing.assert_allclose(s.residual_l2(), aref.hist_l2, rtol=1e-8)
    sm = mg.Solver(p.psi, N, precision=mg.PREC_MIXED)
    um, hm = sm.solve(p.f, p.g, tol=1e-10)
    l2m = sm.residual_l2()
    assert len(l2m) == len(hm) and l2m[0] == pytest.approx(ref.hist_l2[0], rel=1e-12)
    assert l2m[-1] <= 1e-9 * l2m[0]


@pytest.mark.parametrize("reverse", [False, True], ids=["forward", "transposed"])
def test_single_steps_on_the_levels_of_n1024(reverse):
    """One smoothing step on levels 1-4 of the flower at N = 1024 (512 ... 64
    cells per side: the 64 x 16 and 16 x 16 sweep tiles and the cut-vertex
    groups of grids larger than the N = 128 case), from random data, against
    the oracle's smoothing step."""
    mg = _gpu()
    p, d, H = oracle_for("flower", 1024)
    s = mg.Solver(p.psi, 1024)
    for level in (1, 2, 3, 4):
        lv = H.levels[level]
        rng = np.random.default_rng(10 + level)
        x0 = rng.standard_normal(lv.A.shape[0]) * lv.active
        b = rng.standard_normal(lv.A.shape[0]) * lv.active
        xo = x0.copy()
        omg.smoothing_step(lv, xo, b, 4, reverse=reverse)
        xg = torch.tensor(x0, device="cuda:0")
        s.smooth(level, xg, torch.tensor(b, device="cuda:0"), 1, reverse)
        assert rel_max(xg.cpu().numpy(), xo) < 1e-13, level
