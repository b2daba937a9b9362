"""Oracle adjoint of the multigrid solve (test infrastructure).

Misfit J(u) = 1/2 int_Omega (u - u_t)^2, with u and u_t replaced by their
nodal Q1 interpolants so that J = 1/2 e^T M e, e = u - u_t, and
dJ/du = M e (a reading: the objective is not part of the paper).

The forward solver maps the data linearly to the k-th iterate,
u_k = B_k F with F = M f + G g.  Its exact discrete adjoint applies B_k^T,
which is k cycles of the transposed cycle from a zero guess: every smoothing
phase in reverse order and the pre/post smoothing counts swapped (the Galerkin
coarse correction with R = P^T is self-adjoint in the A inner product, and
A = A^T).  Then dJ/df = M^T lam = M lam, dJ/dg = G^T lam and, with Neumann
segments, dJ/dg_N = GN^T lam.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import multigrid as mg


def misfit(disc, u, ut):
    """J = 1/2 (u - u_t)^T M (u - u_t) and dJ/du = M (u - u_t)."""
    e = u - ut
    Me = disc.M @ e
    return 0.5 * float(e @ Me), Me


def adjoint_solve(hier, dJdu, tol=1e-10, max_cycles=50, nu1=2, nu2=1, eta=4):
    """lam from the transposed cycle applied to dJ/du."""
    return mg.solve(hier, dJdu, tol=tol, max_cycles=max_cycles, nu1=nu2, nu2=nu1,
                    eta=eta, reverse=True)


def gradients(disc, lam):
    """(dJ/df, dJ/dg) = (M lam, G^T lam)."""
    return disc.M @ lam, disc.G.T @ lam


def neumann_gradient(disc, lam):
    """dJ/dg_N = GN^T lam (GN symmetric); zero without Neumann segments."""
    if disc.GN is None:
        return np.zeros(disc.n)
    return disc.GN.T @ lam


def forward(hier, disc, f, g, cycles, nu1=2, nu2=1, eta=4):
    """u_k for a fixed number of cycles from zero (a linear map of (f, g))."""
    return mg.solve(hier, disc.rhs(f, g), tol=-1.0, max_cycles=cycles, nu1=nu1,
                    nu2=nu2, eta=eta).u


def dense_adjoint(disc, dJdu):
    """lam = A^{-1} dJ/du on the active nodes by a direct sparse solve."""
    a = np.nonzero(disc.A.diagonal() != 0.0)[0]
    lam = np.zeros(disc.n)
    lam[a] = spla.spsolve(disc.A[a][:, a].tocsc(), dJdu[a])
    return lam
