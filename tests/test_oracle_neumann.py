"""Pins of the oracle's mixed Dirichlet/Neumann boundaries (section 2, eqs.
disc_bil_form and disc_rhs: no penalty or Nitsche terms on Gamma_N, the load
int g_N v there; section 5.3, the annulus and the leaf).

  * Consistency: a linear u lies in the Q1 space and meets the Neumann data
    exactly on a straight Neumann side, so the discrete solution is u itself
    (vertical and horizontal strips, a tilted rectangle).  The Dirichlet data
    are wrong by 5 where only Neumann cells read them, so a segment taken for
    the wrong part of the boundary shows.
  * Without an indicator the assembly is the Dirichlet one; with Neumann
    segments everywhere the operator annihilates constants and GN sums to
    the length of the discrete boundary.
  * Second-order convergence on the annulus and the leaf (the order the
    paper states for the ghost-FEM) with a snapping exponent of 2.5; the
    default 1.75 moves boundary nodes by h^1.75 and bends the Neumann side
    there, which limits the order on Gamma_N to about 1.75.
  * The two-grid factors of section 5.3 (gamma = 2, eta = 4) on the annulus
    and the leaf, and dJ/dg_N against finite differences.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import adjoint as oadj
from oracle import assembly as oasm
from oracle import geometry as geo
from oracle import multigrid as omg


def _direct(d, F):
    a = np.nonzero(d.active)[0]
    u = np.zeros(d.n)
    u[a] = spla.spsolve(d.A[a][:, a].tocsc(), F[a])
    return u


@pytest.mark.parametrize("N", [32, 64, 128])
@pytest.mark.parametrize("case", ["strip_x", "strip_y", "rectangle"])
def test_linear_solution_reproduced(case, N):
    p = {"strip_x": lambda: W.linear_strip(N, axis=0),
         "strip_y": lambda: W.linear_strip(N, axis=1),
         "rectangle": lambda: W.linear_rectangle(N)}[case]()
    d = oasm.assemble(p.psi, N, chi=p.chi)
    assert d.GN.nnz > 0
    u = _direct(d, d.rhs(p.f, p.g, p.gN))
    assert np.abs(u - p.u_exact)[d.active].max() < 1e-10


def test_no_indicator_is_the_dirichlet_assembly():
    N = 64
    p = W.flower_mms(N)
    d0 = oasm.assemble(p.psi, N)
    d1 = oasm.assemble(p.psi, N, chi=-np.ones(d0.n))
    assert d0.GN is None
    assert np.all(d1.GN.data == 0.0)
    for X, Y in ((d0.A, d1.A), (d0.M, d1.M), (d0.G, d1.G)):
        assert (X != Y).nnz == 0
    assert np.array_equal(d0.cell_lambda, d1.cell_lambda)


@pytest.mark.parametrize("N", [64, 128])
def test_all_neumann_circle(N):
    """chi > 0 everywhere: A annihilates constants, G and lambda vanish, and
    1^T GN 1 is the length of the discrete boundary, 2 pi r + O(h^2)."""
    r = 0.55
    psi = W.circle(N, radius=r)
    d = oasm.assemble(psi, N, chi=np.ones((N + 1) ** 2))
    one = d.active.astype(float)
    assert np.abs(d.A @ one).max() < 1e-12
    assert np.abs(d.G.data).max() == 0.0
    assert np.all(d.cell_lambda == 0.0)
    length = float(one @ (d.GN @ one))
    # the discrete boundary: the segment lengths of every cut cell
    segs = 0.0
    psi4 = geo.cell_vertex_values(d.psi, N)
    for c in d.cut_cells:
        for P, Q in geo.cut_geometry(psi4[c])[2]:
            segs += math.hypot(Q[0] - P[0], Q[1] - P[1]) * d.h
    assert length == pytest.approx(segs, rel=1e-12)
    assert abs(length - 2 * math.pi * r) < 2.0 * d.h ** 2


@pytest.mark.parametrize("name", ["annulus", "leaf"])
def test_second_order_convergence(name):
    gen = {"annulus": W.annulus_mms, "leaf": W.leaf_mms}[name]
    errs = []
    for N in (64, 128, 256):
        p = gen(N)
        d = oasm.assemble(p.psi, N, chi=p.chi, alpha=2.5)
        u = _direct(d, d.rhs(p.f, p.g, p.gN))
        errs.append(np.abs(u - p.u_exact)[p.psi < 0].max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.85), rates


@pytest.mark.parametrize("name", ["annulus", "leaf"])
def test_two_grid_factor_mixed_boundaries(name):
    """h = 2^-5 on [-1, 1]^2 (N = 64), gamma = 2: with eta = 4 the two-grid
    factor is at most about 0.1 (section 5.3); without the extra sweeps it is
    several times larger."""
    p = {"annulus": W.annulus_mms, "leaf": W.leaf_mms}[name](64)
    d = oasm.assemble(p.psi, 64, chi=p.chi)
    H2 = omg.two_grid(d)
    rho4 = omg.rho_protocol(H2, eta=4)
    rho0 = omg.rho_protocol(H2, eta=0)
    assert rho4 < 0.12
    assert rho0 > 3 * rho4


def test_rediscretised_hierarchy_with_neumann():
    """Coarse levels assembled on their own grids with chi injected like psi:
    the V-cycle converges to the direct solution of the fine problem."""
    N = 128
    p = W.annulus_mms(N)
    d = oasm.assemble(p.psi, N, chi=p.chi)
    H = omg.build_hierarchy(d, rediscretise=(p.psi, {"chi": p.chi}))
    assert H.levels[1].A.nnz > 0
    F = d.rhs(p.f, p.g, p.gN)
    res = omg.solve(H, F, tol=1e-11, max_cycles=60)
    assert res.converged
    u = _direct(d, F)
    assert np.abs(res.u - u).max() < 1e-8 * np.abs(u).max()


def test_neumann_gradient_finite_differences():
    """dJ/dg_N = GN^T lam with lam = A^-1 M (u - u_t): J is quadratic in g_N,
    so central differences agree to rounding."""
    N = 32
    p = W.annulus_mms(N)
    d = oasm.assemble(p.psi, N, chi=p.chi)
    ut = W.adjoint_target(N)

    def J(gN):
        u = _direct(d, d.rhs(p.f, p.g, gN))
        return oadj.misfit(d, u, ut)[0]

    u = _direct(d, d.rhs(p.f, p.g, p.gN))
    _, dJdu = oadj.misfit(d, u, ut)
    lam = oadj.dense_adjoint(d, dJdu)
    grad = oadj.neumann_gradient(d, lam)
    assert np.abs(grad).max() > 0
    for v in W.random_directions(d.n, 4, seed=3):
        eps = 1e-3
        fd = (J(p.gN + eps * v) - J(p.gN - eps * v)) / (2 * eps)
        assert float(grad @ v) == pytest.approx(fd, rel=1e-7)
