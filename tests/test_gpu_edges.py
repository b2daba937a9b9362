"""GPU edge cases: domains that reach the sides of the box (sweep tiles whose
staged region crosses the grid's sides), grids whose coarsest level is not
4 x 4 (N = coarsest_n 2^k with coarsest_n in {3, 5, 12}: ragged tiles on every
level) against the oracle, and the largest grid of these tests, N = 8192 (67M
nodes), where the oracle is too slow and properties stand in.
"""
import numpy as np
import pytest

import workloads as W
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


@pytest.mark.parametrize("N,center,radius", [(256, (0.0, -0.03), 0.985), (512, (0.004, -0.03), 0.99)])
def test_domains_at_the_box_sides(N, center, radius):
    """Circles that reach the sides of the box, so that the staged regions of
    the sweep tiles cross the grid's sides on every sweep level, with the first
    active column at 3 and 1 (N = 512, 256) or 0: the groups of 16 bytes that
    straddle a side (two float64 or four float32 nodes, also those of the
    coarse tile of a fused prolongation) are filled in node by node.  Iterates
    after 3 cycles and the converged solution against the oracle; the mixed
    form (float32 sweeps) to the float64 tolerance, at the oracle's solution."""
    mg = _gpu()
    rng = np.random.default_rng(N)
    psi = W.circle(N, radius=radius, center=center)
    d = oasm.assemble(psi, N)
    H = omg.build_hierarchy(d)
    f = rng.uniform(-1, 1, d.n)
    g = rng.uniform(-1, 1, d.n)
    F = d.rhs(f, g)
    s = mg.Solver(psi, N)
    act = s.export(mg._lib.EXPORT_NODE_FLAGS).cpu().numpy().astype(int).reshape(N + 1, N + 1) & 1
    assert act[:, 0].any() or act[:, 1].any() or act[:, 3].any()
    u, _ = s.solve(f, g, tol=-1.0, max_cycles=3)
    ref = omg.solve(H, F, tol=-1.0, max_cycles=3)
    assert rel_max(u.cpu().numpy(), ref.u) < 1e-10
    u, hist = s.solve(f, g, tol=1e-10, max_cycles=60)
    ref = omg.solve(H, F, tol=1e-10, max_cycles=60)
    assert s.last_status == 0 and ref.converged and len(hist) == len(ref.hist)
    assert rel_max(u.cpu().numpy(), ref.u) < 1e-10
    sm = mg.Solver(psi, N, precision=mg.PREC_MIXED, inner_cycles=1)
    um, hm = sm.solve(f, g, tol=1e-10, max_cycles=60)
    assert sm.last_status == 0 and hm[-1] <= 1e-10 * np.abs(F).max()
    assert rel_max(um.cpu().numpy(), ref.u) < 1e-8


@pytest.mark.parametrize("cn,k", [(3, 5), (5, 6), (12, 3), (3, 9)])
def test_other_coarsest_sizes(cn, k):
    mg = _gpu()
    N = cn * 2 ** k
    p = W.flower_mms(N)
    d = oasm.assemble(p.psi, N)
    H = omg.build_hierarchy(d, coarsest_n=cn)
    F = d.rhs(p.f, p.g)
    s = mg.Solver(p.psi, N, coarsest_n=cn)
    assert s.n_levels == len(H.levels)
    assert s.level_n(s.n_levels - 1) == cn
    u, hist = s.solve(p.f, p.g, tol=-1.0, max_cycles=3)
    ref = omg.solve(H, F, tol=-1.0, max_cycles=3)
    # the bar of the full-size tests: rounding grows with the number of levels
    assert rel_max(u.cpu().numpy(), ref.u) < 1e-10
    np.testing.assert_allclose(hist, ref.hist, rtol=1e-8, atol=50 * 2.2e-16 * hist[0])


def test_largest_grid_converges():
    """N = 8192: the solve reaches the tolerance with a decreasing residual,
    inactive nodes stay zero, and the solution agrees with the N = 4096 one at
    the shared nodes and with the manufactured solution to 1e-4.  (At these
    sizes the max-norm error against the manufactured solution no longer
    falls like h^2: it is about 1e-5 at both sizes, and at N = 4096 the
    oracle's solution, which the full-size tests match to 1e-10, has the
    same error.)"""
    mg = _gpu()
    sol = {}
    for N in (4096, 8192):
        p = W.flower_mms(N)
        s = mg.Solver(p.psi, N)
        u, hist = s.solve(p.f, p.g, tol=1e-10, max_cycles=60)
        assert s.last_status == 0 and hist[-1] <= 1e-10 * hist[0]
        assert np.all(np.diff(hist) < 0)
        ug = u.cpu().numpy()
        inside = p.psi < 0
        active = (s.export(mg._lib.EXPORT_NODE_FLAGS).cpu().numpy().astype(int) & 1) == 1
        assert np.all(ug[~active] == 0)
        assert np.abs(ug - p.u_exact)[inside].max() < 1e-4
        sol[N] = (ug.reshape(N + 1, N + 1), inside.reshape(N + 1, N + 1))
        s.close()
        del u
        torch.cuda.empty_cache()
    coarse, cin = sol[4096]
    fine, fin = sol[8192]
    both = cin & fin[::2, ::2]
    assert np.abs(coarse - fine[::2, ::2])[both].max() < 1e-4
