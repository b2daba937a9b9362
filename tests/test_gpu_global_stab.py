"""GPU parity of the global stabilisation parameter (section 5.2: lambda =
gamma C on every cut cell, C the largest eigenvalue of K v = Lambda S v),
computed at setup by Lanczos iterations with multigrid solves for S, against
the oracle's direct generalised eigensolver: C, the closed form of the box cut
by a vertical line, the assembled operator, and the two-grid factors of the
paper's circle (section 5.3), where the global parameter converges worse than
the local one.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assembly as oasm
from oracle import geometry as geo
from oracle import multigrid as omg

from helpers import planes_from_csr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_05105_amd as mg
    return mg


def _oracle_C(psi, N, box, chi=None):
    h = (box[2] - box[0]) / N
    psi4 = geo.cell_vertex_values(geo.snap(psi, h, 1.75), N)
    chi4 = None if chi is None else geo.cell_vertex_values(chi, N)
    return oasm.global_eigen_constant(psi4, geo.classify(psi4), N, h, chi4)


def _solver(mg, psi, N, box, **kw):
    return mg.Solver(psi, N, x_lo=box[0], y_lo=box[1], x_hi=box[2], y_hi=box[3], **kw)


@pytest.mark.parametrize("theta", [0.3, 0.7])
def test_vertical_line_closed_form_on_gpu(theta):
    mg = _gpu()
    N = 64
    s = _solver(mg, W.vertical_line(N, theta), N, W.UNIT_BOX, stab_rule=mg.STAB_GLOBAL)
    inf = s.info()
    assert inf["global_C"] == pytest.approx(N / theta, rel=1e-9)
    assert inf["global_iters"] > 0


@pytest.mark.parametrize("name,N", [("circle", 64), ("flower", 128), ("flower", 1024)])
def test_global_constant_matches_oracle(name, N):
    mg = _gpu()
    if name == "circle":
        box, psi = W.UNIT_BOX, W.circle_quadratic(N)
    else:
        box, psi = W.BOX, W.flower(N)
    C = _oracle_C(psi, N, box)
    s = _solver(mg, psi, N, box, stab_rule=mg.STAB_GLOBAL)
    inf = s.info()
    assert inf["global_C"] == pytest.approx(C, rel=1e-8), inf["global_iters"]
    lam = s.export(mg._lib.EXPORT_CELL_LAMBDA).cpu().numpy()
    ct = s.export(mg._lib.EXPORT_CELL_TYPE).cpu().numpy()
    cut = (ct != 0) & (ct != 4)
    assert np.all(lam[cut] == 2.0 * inf["global_C"])
    if N <= 128:
        d = oasm.assemble(psi, N, box=box, rule=geo.STAB_GLOBAL)
        got = s.export(mg._lib.EXPORT_A).cpu().numpy().reshape(9, -1)
        ref = planes_from_csr(d.A, N)
        assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


def test_global_constant_with_neumann_segments():
    mg = _gpu()
    N = 128
    p = W.annulus_mms(N)
    C = _oracle_C(p.psi, N, W.BOX, p.chi)
    s = mg.Solver(p.psi, N, chi=p.chi, stab_rule=mg.STAB_GLOBAL)
    assert s.info()["global_C"] == pytest.approx(C, rel=1e-8)


def test_global_rule_two_grid_factors():
    """Circle r = 0.4 in [0,1]^2, N = 64, gamma = 2: the GPU factors with the
    global parameter are the oracle's and larger than the local ones."""
    mg = _gpu()
    N = 64
    box = W.UNIT_BOX
    psi = W.circle_quadratic(N)
    n = (N + 1) ** 2
    z = np.zeros(n)
    rho = {}
    for rule in (mg.STAB_LOCAL_EIG, mg.STAB_GLOBAL):
        for eta in (0, 4):
            s = _solver(mg, psi, N, box, stab_rule=rule, eta=eta, cycle=mg.CYCLE_TWO_GRID)
            _, hist = s.solve(z, z, tol=-1.0, max_cycles=30, u0=np.ones(n))
            rho[rule, eta] = float(np.mean((hist[1:] / hist[:-1])[20:30]))
            s.close()
    d = oasm.assemble(psi, N, box=box, rule=geo.STAB_GLOBAL)
    H2 = omg.two_grid(d)
    assert abs(rho[mg.STAB_GLOBAL, 0] - omg.rho_protocol(H2, eta=0)) < 0.02
    assert abs(rho[mg.STAB_GLOBAL, 4] - omg.rho_protocol(H2, eta=4)) < 0.02
    assert rho[mg.STAB_GLOBAL, 0] > rho[mg.STAB_LOCAL_EIG, 0] + 0.1
    assert rho[mg.STAB_GLOBAL, 4] > rho[mg.STAB_LOCAL_EIG, 4]


def test_global_rule_parameter_checks():
    mg = _gpu()
    p = W.circle_mms(64)
    with pytest.raises(mg.MgfemError):
        mg.Solver(p.psi, 64, stab_rule=mg.STAB_GLOBAL, coarse_op=mg.COARSE_REDISCRETISED)
    with pytest.raises(mg.MgfemError):
        mg.Solver(p.psi, 64, stab_rule=4)
