"""Oracle quadrature: exact integration of Q1 basis products (test infrastructure).

The paper computes its integrals with Gridap and does not state the rules.
Reading: every cut-cell integral is exact.  Stiffness integrands are of
degree 2 and mass integrands of degree 4 on the polygon; on the interface
segment the Nitsche integrand (n . grad phi_j) phi_i is cubic and the penalty
integrand phi_i phi_j quartic in the arc parameter.  The rules below
(Gauss-Legendre on the collapsed square for triangles, fan triangulation for
polygons, Gauss-Legendre on segments) are exact well beyond those degrees.
"""
from __future__ import annotations

import numpy as np


def gauss01(n):
    """n-point Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_rule(a, b, c, n=4):
    """Collapsed-coordinate (Duffy) Gauss rule on triangle abc.

    x(s, t) = a + s (b - a) + s t (c - b), Jacobian s |det(b - a, c - b)|.
    With n points per direction it integrates total degree 2n - 2 exactly."""
    s, ws = gauss01(n)
    t, wt = gauss01(n)
    S, T = np.meshgrid(s, t, indexing="ij")
    W = np.outer(ws, wt)
    a, b, c = (np.asarray(v, dtype=np.float64) for v in (a, b, c))
    jac = abs((b[0] - a[0]) * (c[1] - b[1]) - (b[1] - a[1]) * (c[0] - b[0]))
    pts = a[None, :] + S.ravel()[:, None] * (b - a)[None, :] \
        + (S * T).ravel()[:, None] * (c - b)[None, :]
    return pts, (W * S).ravel() * jac


def polygon_rule(poly, n=4):
    """Fan triangulation of a convex-or-star polygon from its first vertex."""
    pts, wts = [], []
    for i in range(1, len(poly) - 1):
        p, w = triangle_rule(poly[0], poly[i], poly[i + 1], n)
        pts.append(p)
        wts.append(w)
    return np.concatenate(pts), np.concatenate(wts)


def segment_rule(P, Q, n=3):
    """Gauss-Legendre on segment PQ (exact to degree 2n - 1)."""
    t, w = gauss01(n)
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    length = float(np.hypot(*(Q - P)))
    return P[None, :] + t[:, None] * (Q - P)[None, :], w * length


def q1_basis(pts):
    """Q1 basis on the reference cell at points (m, 2): returns (4, m)."""
    x, y = pts[:, 0], pts[:, 1]
    return np.stack([(1 - x) * (1 - y), x * (1 - y), x * y, (1 - x) * y])


def q1_grad(pts):
    """Reference gradients of the Q1 basis: returns (4, m, 2)."""
    x, y = pts[:, 0], pts[:, 1]
    gx = np.stack([-(1 - y), (1 - y), y, -y])
    gy = np.stack([-(1 - x), -x, x, (1 - x)])
    return np.stack([gx, gy], axis=-1)
