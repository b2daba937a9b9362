"""Oracle geometry: snapping, cut-cell classification, cut polygons, C(K).

Test infrastructure (see the package docstring); never used by the product path.

All per-cell work is done in the reference cell [0,1]^2 with the four vertices
numbered counter-clockwise,

    v0 = (0,0), v1 = (1,0), v2 = (1,1), v3 = (0,1),

so that cell (i, j) of an N x N grid has global vertices
k(i,j), k(i+1,j), k(i+1,j+1), k(i,j+1) with k(i,j) = i + j (N+1).
Edge e runs from v_e to v_{(e+1) mod 4}.

Cell type codes (shared convention with the HIP path, implemented separately):
    0 external, 1 triangle, 2 quadrilateral, 3 pentagon, 4 internal,
    5 saddle split into two triangles, 6 saddle joined into a hexagon.
"""
from __future__ import annotations

import math

import numpy as np

EXTERNAL, TRIANGLE, QUAD, PENTAGON, INTERNAL, SADDLE_SPLIT, SADDLE_HEX = range(7)

REF_VERTS = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])

STAB_PAPER, STAB_LOCAL_EIG, STAB_FIXED, STAB_GLOBAL = 0, 1, 2, 3


# ----------------------------------------------------------------------------
# Snapping back to grid (section 2)
# ----------------------------------------------------------------------------

def snap(psi: np.ndarray, h: float, alpha: float) -> np.ndarray:
    """Snapping-back-to-grid (section 2): a node inside the domain (psi < 0)
    with |psi| < h**alpha gets psi := 0.  Nodes with psi >= 0 are untouched.
    The exponent is positive (the definition in section 2; the 1D test text's
    negative sign is read as a typo)."""
    out = np.array(psi, dtype=np.float64, copy=True)
    out[(out < 0.0) & (np.abs(out) < h ** alpha)] = 0.0
    return out


def cell_vertex_values(psi: np.ndarray, N: int) -> np.ndarray:
    """(N*N, 4) array of nodal values at v0..v3 of every cell, cell index
    c = ci + cj N."""
    P = psi.reshape(N + 1, N + 1)  # P[j, i]
    return np.stack([P[:-1, :-1], P[:-1, 1:], P[1:, 1:], P[1:, :-1]], axis=-1).reshape(N * N, 4)


def classify(psi4: np.ndarray) -> np.ndarray:
    """Cell type from the signs of psi at its vertices (section 5.2): a vertex
    is internal iff psi < 0 (psi == 0 counts as external).  One internal vertex
    gives a triangle, two adjacent a quadrilateral, three a pentagon.  Two
    diagonal internal vertices (a saddle, not covered by the paper) are split
    or joined by the sign of the mean of the four values: mean >= 0 gives two
    triangles, mean < 0 a hexagon."""
    psi4 = np.atleast_2d(psi4)
    inside = psi4 < 0.0
    k = inside.sum(axis=1)
    t = np.full(len(psi4), EXTERNAL, dtype=np.int64)
    t[k == 1] = TRIANGLE
    t[k == 3] = PENTAGON
    t[k == 4] = INTERNAL
    two = k == 2
    diag = two & (inside[:, 0] == inside[:, 2])
    t[two & ~diag] = QUAD
    mean_neg = psi4.mean(axis=1) < 0.0
    t[diag & mean_neg] = SADDLE_HEX
    t[diag & ~mean_neg] = SADDLE_SPLIT
    return t


def _edge_cuts(psi4):
    """Cut points on the edges whose end vertices differ in sign class.

    Returns {edge: (point, theta, internal_vertex)} where theta is the cut
    fraction measured from the internal vertex by linear interpolation of psi
    along the edge (section 5.2): theta = psi_in / (psi_in - psi_out)."""
    inside = psi4 < 0.0
    cuts = {}
    for e in range(4):
        a, b = e, (e + 1) % 4
        if inside[a] != inside[b]:
            p, q = (a, b) if inside[a] else (b, a)
            th = psi4[p] / (psi4[p] - psi4[q])
            cuts[e] = (REF_VERTS[p] + th * (REF_VERTS[q] - REF_VERTS[p]), float(th), p)
    return cuts


def cut_geometry(psi4):
    """Polygon(s) K cap Omega and interface segment(s) Gamma cap K of one cell,
    in reference coordinates.

    Returns (type, polygons, segments, cuts) where polygons is a list of
    (m, 2) arrays listed counter-clockwise, segments a list of (P, Q) pairs
    oriented so that the polygon lies on their left (the outward normal of
    Omega is the right-hand normal of P -> Q), and cuts the edge-cut map."""
    psi4 = np.asarray(psi4, dtype=np.float64)
    t = int(classify(psi4[None, :])[0])
    inside = psi4 < 0.0
    if t == EXTERNAL:
        return t, [], [], {}
    if t == INTERNAL:
        return t, [REF_VERTS.copy()], [], {}
    cuts = _edge_cuts(psi4)
    if t == SADDLE_SPLIT:
        polys, segs = [], []
        for p in range(4):
            if inside[p]:
                c_next = cuts[p][0]          # on edge p (v_p -> v_{p+1})
                c_prev = cuts[(p - 1) % 4][0]  # on edge p-1 (v_{p-1} -> v_p)
                polys.append(np.array([REF_VERTS[p], c_next, c_prev]))
                segs.append((c_next, c_prev))
        return t, polys, segs, cuts
    # connected piece: walk the boundary counter-clockwise
    poly, events = [], []
    for e in range(4):
        a, b = e, (e + 1) % 4
        if inside[a]:
            poly.append(REF_VERTS[a])
        if e in cuts:
            poly.append(cuts[e][0])
            events.append(("exit" if inside[a] else "entry", cuts[e][0]))
    segs = []
    n = len(events)
    for idx, (kind, pt) in enumerate(events):
        if kind == "exit":
            for step in range(1, n + 1):
                k2, q = events[(idx + step) % n]
                if k2 == "entry":
                    segs.append((pt, q))
                    break
    return t, [np.array(poly)], segs, cuts


# ----------------------------------------------------------------------------
# Stabilisation constant C(K) (section 5.2)
# ----------------------------------------------------------------------------

def c_triangle(t1, t2, h=1.0):
    """Eq. c_triangle: lower bound of C for a triangular cut region with cut
    sides t1 h and t2 h, written as printed in the paper."""
    num = math.sqrt((t1 ** 2 + t2 ** 2) / t1 ** 2) * (
        3 * t1 ** 4 + 3 * t2 ** 4 + math.sqrt(3 * (t1 ** 8 + 10 * t1 ** 4 * t2 ** 4 + t2 ** 8)))
    return num / (h * t2 * (t1 ** 2 + t2 ** 2) ** 2)


def c_pentagon(h=1.0):
    """Eq. c_pentagon: 3 sqrt(2) / h, the triangle value at t1 = t2 = 1."""
    return 3.0 * math.sqrt(2.0) / h


def c_quadrilateral(t1, t2, h=1.0):
    """The quadrilateral bound of section 5.2, C = (3 h L Q + sqrt(3 h^2 P)) / (h^2 D).

    The printed formula is garbled by line breaks (a stray '2 *', one surplus
    closing parenthesis after the t1^8 group, and the '- t1^2(-1 + 2 t2^2 +
    t2^4)' term broken out of its bracket).  Reading: the surplus parenthesis
    is dropped and the broken-out term belongs to the first polynomial Q.
    This reading is checked against the local eigenproblem in the tests."""
    L = math.sqrt(1 + t1 ** 2 - 2 * t1 * t2 + t2 ** 2)
    Q = (t1 ** 6 + 2 * t1 ** 3 * t2 + t2 ** 2 - t1 ** 4 * t2 ** 2 + t2 ** 6
         + 2 * t1 * (t2 + t2 ** 3) - t1 ** 2 * (-1 + 2 * t2 ** 2 + t2 ** 4))
    P = (t1 ** 14 + 2 * t1 ** 13 * t2 + t1 ** 12 * (1 - 5 * t2 ** 2)
         - 4 * t1 ** 11 * t2 * (-4 + 7 * t2 ** 2)
         - 2 * t1 ** 9 * t2 * (-6 + 20 * t2 ** 2 + 17 * t2 ** 4)
         + t1 ** 10 * (10 - 22 * t2 ** 2 + 73 * t2 ** 4)
         + t1 ** 8 * (10 - 38 * t2 ** 2 + 63 * t2 ** 4 - 69 * t2 ** 6)
         + 8 * t1 ** 7 * t2 * (4 - 4 * t2 ** 2 + 3 * t2 ** 4 + 15 * t2 ** 6)
         + t1 ** 6 * (1 - 32 * t2 ** 2 + 136 * t2 ** 4 - 84 * t2 ** 6 - 69 * t2 ** 8)
         + 2 * t1 * t2 ** 5 * (5 + 16 * t2 ** 2 + 6 * t2 ** 4 + 8 * t2 ** 6 + t2 ** 8)
         - 4 * t1 ** 3 * t2 ** 3 * (5 + 14 * t2 ** 2 + 8 * t2 ** 4 + 10 * t2 ** 6 + 7 * t2 ** 8)
         - 2 * t1 ** 5 * t2 * (-5 + 28 * t2 ** 2 + 88 * t2 ** 4 - 12 * t2 ** 6 + 17 * t2 ** 8)
         + t2 ** 4 * (1 + t2 ** 2 + 10 * t2 ** 4 + 10 * t2 ** 6 + t2 ** 8 + t2 ** 10)
         - t1 ** 2 * t2 ** 2 * (2 + t2 ** 2 + 32 * t2 ** 4 + 38 * t2 ** 6 + 22 * t2 ** 8 + 5 * t2 ** 10)
         + t1 ** 4 * (1 - t2 ** 2 + 104 * t2 ** 4 + 136 * t2 ** 6 + 63 * t2 ** 8 + 73 * t2 ** 10))
    D = (t1 ** 7 + t1 ** 6 * t2 + t1 ** 5 * (2 - 3 * t2 ** 2) + t1 ** 3 * (-1 + t2 ** 2) ** 2
         + t2 ** 3 * (1 + t2 ** 2) ** 2 + t1 ** 4 * t2 * (6 + t2 ** 2)
         + t1 * t2 ** 2 * (5 + 6 * t2 ** 2 + t2 ** 4) + t1 ** 2 * (5 * t2 - 2 * t2 ** 3 - 3 * t2 ** 5))
    return (3 * h * L * Q + math.sqrt(3 * h ** 2 * P)) / (h ** 2 * D)


def cut_fractions(t, cuts, psi4):
    """The (theta1, theta2) pairs that enter C(K) for a cut cell.

    Triangle: the two cut fractions measured from the internal vertex.
    Quadrilateral: the fraction on each cut edge, each measured from its own
    internal vertex (figure cut_geos).  Saddle split: one pair per triangle."""
    inside = psi4 < 0.0
    if t in (TRIANGLE, SADDLE_SPLIT):
        pairs = []
        for p in range(4):
            if inside[p]:
                pairs.append((cuts[p][1], cuts[(p - 1) % 4][1]))
        return pairs
    if t == QUAD:
        return [tuple(cuts[e][1] for e in sorted(cuts))]
    return []


def stabilization_constant(psi4, h=1.0, rule=STAB_PAPER, geometry=None):
    """C(K) for one cut cell by the paper's closed forms (rule STAB_PAPER):
    triangle eq. c_triangle, quadrilateral formula, pentagon eq. c_pentagon.
    Saddle cells: the larger of the two triangle values when split, the
    pentagon value when joined into a hexagon.  Rule STAB_LOCAL_EIG solves the
    local 4x4 generalised eigenproblem of section 5.2 instead."""
    psi4 = np.asarray(psi4, dtype=np.float64)
    t, polys, segs, cuts = geometry if geometry is not None else cut_geometry(psi4)
    if rule == STAB_LOCAL_EIG:
        from .assembly import local_eigen_constant
        return local_eigen_constant(polys, segs) / h
    if t in (TRIANGLE, SADDLE_SPLIT):
        return max(c_triangle(a, b, h) for a, b in cut_fractions(t, cuts, psi4))
    if t == QUAD:
        (a, b), = cut_fractions(t, cuts, psi4)
        return c_quadrilateral(a, b, h)
    if t in (PENTAGON, SADDLE_HEX):
        return c_pentagon(h)
    return 0.0


def polygon_area(poly):
    """Shoelace area of a counter-clockwise polygon."""
    x, y = poly[:, 0], poly[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))
