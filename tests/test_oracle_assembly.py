"""Pins of the oracle's ghost-FEM assembly (CPU only): exact Q1 integrals,
conservation identities, exactness on bilinear functions (consistency of the
Nitsche form), symmetry/definiteness and second-order convergence on
manufactured solutions (section 2, eqs. disc_bil_form / disc_rhs)."""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import assembly as asm
from oracle import geometry as geo


def test_polygon_quadrature_reproduces_closed_form_q1_matrices():
    S, M, B, L, Kn = asm.reference_integrals([geo.REF_VERTS], [])
    S_int, M_int = asm.interior_matrices(1.0)
    np.testing.assert_allclose(S, S_int, atol=1e-15)
    np.testing.assert_allclose(M, M_int, atol=1e-15)


def test_interior_stencils():
    N = 16
    d = asm.assemble(W.circle(N, radius=0.9), N)
    h = 2.0 / N
    k = N // 2 + (N // 2) * (N + 1)  # centre node, deep inside
    row = d.A.getrow(k).toarray().ravel()
    mrow = d.M.getrow(k).toarray().ravel()
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            kk = k + di + dj * (N + 1)
            if di == 0 and dj == 0:
                assert row[kk] == pytest.approx(8.0 / 3.0, abs=1e-15)
                assert mrow[kk] == pytest.approx(4 * h * h / 9, rel=1e-14)
            else:
                assert row[kk] == pytest.approx(-1.0 / 3.0, abs=1e-15)
                w = 1.0 / 9.0 if di == 0 or dj == 0 else 1.0 / 36.0
                assert mrow[kk] == pytest.approx(w * h * h, rel=1e-14)
    assert np.count_nonzero(row) == 9


def _random_cut_cells(rng, count):
    out = []
    while len(out) < count:
        psi4 = rng.uniform(-1, 1, size=4)
        t = geo.classify(psi4[None, :])[0]
        if t not in (geo.EXTERNAL, geo.INTERNAL):
            out.append(psi4)
    return out


def test_cut_cell_identities():
    rng = np.random.default_rng(11)
    h = 0.125
    for psi4 in _random_cut_cells(rng, 60):
        t, polys, segs, _ = geo.cut_geometry(psi4)
        S, M, B, L, _ = asm.reference_integrals(polys, segs)
        area = sum(geo.polygon_area(p) for p in polys)
        length = sum(float(np.hypot(*(Q - P))) for P, Q in segs)
        assert area > 0
        np.testing.assert_allclose(S.sum(axis=1), 0.0, atol=1e-14)   # grad of 1 vanishes
        assert M.sum() == pytest.approx(area, rel=1e-13)                # sum phi_i = 1
        assert L.sum() == pytest.approx(length, rel=1e-13)
        np.testing.assert_allclose(B.sum(axis=1), 0.0, atol=1e-13)     # n . grad 1 = 0
        A_K, M_K, G_K, _, (_, C, lam) = asm.cut_element(psi4, h)
        np.testing.assert_allclose(A_K, A_K.T, atol=1e-13)
        assert lam == pytest.approx(2.0 * C)
        assert M_K.sum() == pytest.approx(area * h * h, rel=1e-13)


@pytest.mark.parametrize("make", [lambda N: W.circle(N), lambda N: W.flower(N),
                                  lambda N: W.ellipse(N)])
def test_exact_for_bilinear_functions(make):
    """Nitsche's form is consistent: for u in Q1 with f = -lap u = 0 and g = u,
    the interpolant solves A u = F exactly.  A dropped or mis-signed boundary
    term in A or in G breaks this."""
    N = 32
    x, y = W.grid_xy(N)
    u = 1.0 + 2.0 * x - 3.0 * y + 0.5 * x * y
    d = asm.assemble(make(N), N)
    F = d.rhs(np.zeros_like(u), u)
    r = (d.A @ (u * d.active) - F)[d.active]
    assert np.abs(r).max() < 1e-12 * np.abs(F).max()


def test_symmetric_positive_definite():
    N = 32
    d = asm.assemble(W.flower(N), N)
    assert abs(d.A - d.A.T).max() == 0.0
    a = np.nonzero(d.active)[0]
    scipy.linalg.cholesky(d.A[a][:, a].toarray())  # raises if not SPD
    np.testing.assert_array_equal(d.A.diagonal() != 0, d.active)


def test_area_and_perimeter_of_the_discrete_domain():
    N = 128
    d = asm.assemble(W.circle(N), N)
    area = float(d.rhs(np.ones(d.n), np.zeros(d.n)).sum())   # 1^T M 1 = |Omega_h|
    assert area == pytest.approx(math.pi * 0.25, rel=2e-3)


def _order(errs, Ns):
    p = np.polyfit(np.log(np.asarray(Ns, float)), np.log(errs), 1)
    return -p[0]


@pytest.mark.parametrize("name", ["circle", "flower"])
def test_second_order_on_manufactured_solutions(name):
    """Second-order accuracy (sections 1, 2 and 6): error ratio ~4 per refinement."""
    import scipy.sparse.linalg as spla
    Ns = [32, 64, 128, 256]
    errs = []
    for N in Ns:
        p = W.circle_mms(N) if name == "circle" else W.flower_mms(N)
        d = asm.assemble(p.psi, N)
        a = np.nonzero(d.active)[0]
        F = d.rhs(p.f, p.g)
        u = np.zeros(d.n)
        u[a] = spla.spsolve(d.A[a][:, a].tocsc(), F[a])
        inside = d.psi < 0
        errs.append(np.abs(u - p.u_exact)[inside].max())
    order = _order(errs, Ns)
    assert 1.8 <= order <= 2.3, (errs, order)
