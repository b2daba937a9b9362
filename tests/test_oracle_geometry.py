"""Pins of the oracle's geometry and stabilisation (CPU only).

Each check compares the oracle with something other than itself: the paper's
special cases of the closed forms, the local generalised eigenproblem that
defines C(K) (section 5.2), hand-computed single-cell configurations.
"""
import math

import numpy as np
import pytest

from oracle import assembly as asm
from oracle import geometry as geo


def tri_psi(t1, t2):
    """psi at v0..v3 with only v0 inside; cut fraction t1 on edge v0-v1 and
    t2 on edge v0-v3 (linear interpolation gives theta = psi0/(psi0 - psi1))."""
    p0 = -1.0
    return np.array([p0, p0 - p0 / t1, 5.0, p0 - p0 / t2])


def quad_psi(t1, t2):
    """v0, v3 inside; fraction t1 on v0-v1 from v0, t2 on v3-v2 from v3."""
    return np.array([-1.0, -1.0 + 1.0 / t1, -1.0 + 1.0 / t2, -1.0])


def pent_psi(t1, t2):
    """v0, v1, v3 inside; fraction t1 on v1-v2 from v1, t2 on v3-v2 from v3.
    v2's value is shared, so t2 is set through v3's value."""
    p2 = 1.0
    p1 = -p2 * t1 / (1.0 - t1)
    p3 = -p2 * t2 / (1.0 - t2)
    return np.array([-1.0, p1, p2, p3])


def test_snap_threshold():
    h, alpha = 0.1, 1.75
    thr = h ** alpha
    psi = np.array([-2 * thr, -0.5 * thr, 0.0, 0.5 * thr, -thr, 1.0])
    out = geo.snap(psi, h, alpha)
    # only nodes inside (psi < 0) and closer than h^alpha are moved to 0
    assert out.tolist() == [-2 * thr, 0.0, 0.0, 0.5 * thr, -thr, 1.0]


@pytest.mark.parametrize("signs,expected", [
    ((1, 1, 1, 1), geo.EXTERNAL),
    ((-1, -1, -1, -1), geo.INTERNAL),
    ((-1, 1, 1, 1), geo.TRIANGLE),
    ((1, 1, -1, 1), geo.TRIANGLE),
    ((-1, -1, 1, 1), geo.QUAD),
    ((1, -1, -1, 1), geo.QUAD),
    ((-1, 1, 1, -1), geo.QUAD),
    ((-1, -1, -1, 1), geo.PENTAGON),
    ((-1, 1, -1, 1), None),   # saddle: decided by the mean
    ((0, 0, 0, 0), geo.EXTERNAL),  # psi == 0 counts as external
    ((-1, 0, 0, 0), geo.TRIANGLE),
])
def test_classify_single_cells(signs, expected):
    psi4 = np.array(signs, dtype=float)
    t = geo.classify(psi4[None, :])[0]
    if expected is None:
        assert t in (geo.SADDLE_SPLIT, geo.SADDLE_HEX)
    else:
        assert t == expected


def test_saddle_split_and_join():
    assert geo.classify(np.array([[-1.0, 2.0, -1.0, 2.0]]))[0] == geo.SADDLE_SPLIT
    assert geo.classify(np.array([[-2.0, 1.0, -2.0, 1.0]]))[0] == geo.SADDLE_HEX
    t, polys, segs, _ = geo.cut_geometry(np.array([-1.0, 2.0, -1.0, 2.0]))
    assert len(polys) == 2 and len(segs) == 2
    t, polys, segs, _ = geo.cut_geometry(np.array([-2.0, 1.0, -2.0, 1.0]))
    assert len(polys) == 1 and len(polys[0]) == 6 and len(segs) == 2


def test_cut_fractions_by_linear_interpolation():
    # triangle at v0: psi0 = -0.3, psi1 = 0.7 -> theta = 0.3 ; psi3 = 0.1 -> 0.75
    psi4 = np.array([-0.3, 0.7, 1.0, 0.1])
    t, polys, segs, cuts = geo.cut_geometry(psi4)
    assert t == geo.TRIANGLE
    assert cuts[0][1] == pytest.approx(0.3)
    assert cuts[3][1] == pytest.approx(0.75)
    assert geo.polygon_area(polys[0]) == pytest.approx(0.5 * 0.3 * 0.75)
    (P, Q), = segs
    # outward normal (right of P -> Q) points away from the inside vertex
    d = Q - P
    n = np.array([d[1], -d[0]])
    assert n @ (0.5 * (P + Q)) > 0


@pytest.mark.parametrize("t1,t2", [(1.0, 1.0), (0.3, 0.7), (0.9, 0.2), (0.05, 0.4), (0.01, 0.02)])
def test_triangle_closed_form_equals_local_eigenproblem(t1, t2):
    psi4 = tri_psi(t1, t2)
    t, polys, segs, _ = geo.cut_geometry(psi4)
    assert t == geo.TRIANGLE
    eig = asm.local_eigen_constant(polys, segs)
    assert geo.c_triangle(t1, t2) == pytest.approx(eig, rel=1e-9)
    assert geo.stabilization_constant(psi4) == pytest.approx(eig, rel=1e-9)


@pytest.mark.parametrize("t1,t2", [(0.5, 0.5), (0.3, 0.7), (0.7, 0.3), (0.05, 0.02), (1.0, 1.0),
                                   (0.9, 0.1), (0.2, 0.95)])
def test_quadrilateral_reading_equals_local_eigenproblem(t1, t2):
    # pins the reading of the garbled quadrilateral formula
    psi4 = quad_psi(t1, t2)
    t, polys, segs, _ = geo.cut_geometry(psi4)
    assert t == geo.QUAD
    eig = asm.local_eigen_constant(polys, segs)
    assert geo.c_quadrilateral(t1, t2) == pytest.approx(eig, rel=1e-9)
    assert geo.c_quadrilateral(t2, t1) == pytest.approx(eig, rel=1e-9)


def test_paper_special_cases():
    # eq. c_pentagon: the triangle formula at t1 = t2 = 1 is 3 sqrt(2) / h
    for h in (1.0, 0.25, 2.0 / 64):
        assert geo.c_triangle(1.0, 1.0, h) == pytest.approx(3 * math.sqrt(2) / h, rel=1e-14)
        assert geo.c_pentagon(h) == pytest.approx(3 * math.sqrt(2) / h, rel=1e-15)
    # rectangle test of section 5.3: equal quadrilateral cuts theta h give C = 1/(theta h)
    for th in (1.0, 0.5, 0.3, 0.01):
        for h in (1.0, 1.0 / 128):
            assert geo.c_quadrilateral(th, th, h) == pytest.approx(1.0 / (th * h), rel=1e-12)


def test_pentagon_value_bounds_pentagon_eigenvalue():
    # section 5.2: pentagons are well posed and the half-cell triangle value suffices
    rng = np.random.default_rng(3)
    for _ in range(40):
        t1, t2 = rng.uniform(0.01, 0.99, size=2)
        t, polys, segs, _ = geo.cut_geometry(pent_psi(t1, t2))
        assert t == geo.PENTAGON
        assert asm.local_eigen_constant(polys, segs) <= geo.c_pentagon() * (1 + 1e-12)


def test_constant_scales_as_inverse_h():
    psi4 = tri_psi(0.3, 0.6)
    assert geo.stabilization_constant(psi4, h=0.5) == pytest.approx(2 * geo.stabilization_constant(psi4, h=1.0))
    assert geo.stabilization_constant(psi4, h=0.5, rule=geo.STAB_LOCAL_EIG) == \
        pytest.approx(geo.stabilization_constant(psi4, h=0.5), rel=1e-9)


def saddle_psi(rng, split):
    """A saddle cell: v0 and v2 inside, v1 and v3 outside; the mean of the
    four values decides between two triangles (>= 0) and one hexagon (< 0)."""
    while True:
        a, c = -rng.uniform(0.05, 2.0, size=2)
        b, d = rng.uniform(0.05, 2.0, size=2)
        if (a + b + c + d >= 0.0) == split:
            return np.array([a, b, c, d])


def _own_segment(poly, segs):
    """The interface segment whose two end points are vertices of poly."""
    for P, Q in segs:
        if all(np.min(np.abs(poly - X).sum(axis=1)) < 1e-14 for X in (P, Q)):
            return P, Q
    raise AssertionError("no segment belongs to this polygon")


def test_split_saddle_constant_is_the_larger_triangle_eigenvalue():
    # reading of saddle cells: split into two triangles, C = max of the two
    # triangle constants; each is checked against the local generalised
    # eigenproblem of section 5.2 posed on that triangle alone, and the
    # eigenproblem of the whole cell (both pieces) stays below it, so
    # lambda_K = gamma C keeps the coercivity bound lambda_K > C_K
    rng = np.random.default_rng(11)
    for _ in range(40):
        psi4 = saddle_psi(rng, split=True)
        t, polys, segs, _ = geo.cut_geometry(psi4)
        assert t == geo.SADDLE_SPLIT and len(polys) == 2 and len(segs) == 2
        each = [asm.local_eigen_constant([p], [_own_segment(p, segs)]) for p in polys]
        C = geo.stabilization_constant(psi4)
        assert C == pytest.approx(max(each), rel=1e-9)
        assert C > min(each) or each[0] == pytest.approx(each[1], rel=1e-9)
        assert asm.local_eigen_constant(polys, segs) <= C * (1 + 1e-12)
        for h in (0.5, 2.0 / 256):
            assert geo.stabilization_constant(psi4, h=h) == pytest.approx(C / h, rel=1e-13)


def test_hexagon_saddle_value_bounds_its_eigenvalue():
    # reading of joined saddle cells: a hexagon takes the pentagon value
    # 3 sqrt(2)/h, which must bound the hexagon's own local eigenvalue
    rng = np.random.default_rng(12)
    for _ in range(40):
        psi4 = saddle_psi(rng, split=False)
        t, polys, segs, _ = geo.cut_geometry(psi4)
        assert t == geo.SADDLE_HEX and len(polys) == 1 and len(polys[0]) == 6
        C = geo.stabilization_constant(psi4)
        assert C == pytest.approx(3 * math.sqrt(2), rel=1e-15)
        assert asm.local_eigen_constant(polys, segs) <= C * (1 + 1e-12)
        # the rule the product also offers: the local eigenproblem itself
        assert geo.stabilization_constant(psi4, rule=geo.STAB_LOCAL_EIG) == \
            pytest.approx(asm.local_eigen_constant(polys, segs), rel=1e-12)
