"""Pins of the global stabilisation parameter (section 5.2: lambda = gamma C
on every cut cell, C the largest eigenvalue of K v = Lambda S v over V_h).

  * Closed form: the unit box cut by the vertical line x = 1 - (1 - theta) h.
    Writing v in the cosine modes of the y direction separates the pencil;
    the mode constant in y gives the largest quotient, and there the problem
    is the 1D chain of edge conductances 1/h (full cells) and theta/h (the
    cut cell) with K = g g^T, g the derivative on the cut cell.  The largest
    quotient puts the whole jump on the cut cell: C = 1 / (theta h).
  * Bounds: e_i^T K e_i / e_i^T S e_i <= C (Rayleigh quotient of a nodal
    basis vector), and C <= max_K C(K) of the local rule (sum the local
    bounds v_K^T K_K v_K <= C(K) v_K^T S_K v_K over the cells).
  * The paper's observation (section 5.3, circular domain): the two-grid
    scheme converges worse with the global parameter than with the local
    one, with and without extra cut-cell sweeps, and the extra sweeps help.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assembly as oasm
from oracle import geometry as geo
from oracle import multigrid as omg


def _pencil_input(psi, N, h):
    ps = geo.snap(psi, h, 1.75)
    psi4 = geo.cell_vertex_values(ps, N)
    return psi4, geo.classify(psi4)


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("theta", [0.3, 0.7])
def test_vertical_line_closed_form(N, theta):
    h = 1.0 / N
    psi4, ct = _pencil_input(W.vertical_line(N, theta), N, h)
    C = oasm.global_eigen_constant(psi4, ct, N, h)
    assert C == pytest.approx(1.0 / (theta * h), rel=1e-12)


@pytest.mark.parametrize("name", ["circle", "flower"])
def test_global_constant_bounds(name):
    if name == "circle":
        N, box, psi = 64, W.UNIT_BOX, W.circle_quadratic(64)
    else:
        N, box, psi = 64, W.BOX, W.flower(64)
    h = (box[2] - box[0]) / N
    psi4, ct = _pencil_input(psi, N, h)
    C = oasm.global_eigen_constant(psi4, ct, N, h)
    K, S, act = oasm.global_pencil(psi4, ct, N, h)
    kd, sd = K.diagonal(), S.diagonal()
    lower = np.max(np.where(act & (sd > 0), kd / np.where(sd > 0, sd, 1.0), 0.0))
    d = oasm.assemble(psi, N, box=box, rule=geo.STAB_LOCAL_EIG)
    upper = d.cell_C[d.cut_cells].max()
    assert lower <= C * (1 + 1e-12)
    assert C <= upper * (1 + 1e-12)
    assert C > 0.2 * upper  # not a degenerate value
    dg = oasm.assemble(psi, N, box=box, rule=geo.STAB_GLOBAL)
    lam = dg.cell_lambda[dg.cut_cells]
    assert np.all(lam == lam[0]) and lam[0] == pytest.approx(2.0 * C, rel=1e-12)


def test_global_parameter_converges_worse_than_local():
    N = 64
    psi = W.circle_quadratic(N)
    rho = {}
    for rule in (geo.STAB_LOCAL_EIG, geo.STAB_GLOBAL):
        d = oasm.assemble(psi, N, box=W.UNIT_BOX, rule=rule)
        H2 = omg.two_grid(d)
        rho[rule] = (omg.rho_protocol(H2, eta=0), omg.rho_protocol(H2, eta=4))
    loc, glo = rho[geo.STAB_LOCAL_EIG], rho[geo.STAB_GLOBAL]
    assert glo[0] > loc[0] + 0.1
    assert glo[1] > loc[1]
    assert glo[1] < glo[0]
