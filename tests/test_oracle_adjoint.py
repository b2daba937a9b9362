"""Pins of the oracle adjoint (CPU only): the transposition identity of the
cycle map, central finite differences of the fixed-cycle solver (exact for the
quadratic misfit up to rounding, because the solver map is linear), and the
direct-solve adjoint."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as adj
from oracle import assembly as asm
from oracle import multigrid as mg


@pytest.fixture(scope="module")
def setup32():
    N = 32
    p = W.flower_mms(N)
    d = asm.assemble(p.psi, N)
    return p, d, mg.build_hierarchy(d)


@pytest.mark.parametrize("k", [1, 3])
def test_transposed_cycle_identity(setup32, k):
    _, d, H = setup32
    rng = np.random.default_rng(2)
    a = rng.standard_normal(d.n) * d.active
    b = rng.standard_normal(d.n) * d.active
    Ba = mg.solve(H, a, tol=-1, max_cycles=k).u
    BTb = adj.adjoint_solve(H, b, tol=-1, max_cycles=k).u
    assert Ba @ b == pytest.approx(a @ BTb, rel=1e-12)
    # the forward cycle itself is not symmetric: the identity is non-trivial
    Bb = mg.solve(H, b, tol=-1, max_cycles=k).u
    assert abs(a @ Bb - a @ BTb) > 1e-8 * abs(a @ BTb)


def test_gradients_match_central_differences(setup32):
    p, d, H = setup32
    k = 6
    ut = W.adjoint_target(d.N)
    u = adj.forward(H, d, p.f, p.g, k)
    J0, dJdu = adj.misfit(d, u, ut)
    lam = adj.adjoint_solve(H, dJdu, tol=-1, max_cycles=k).u
    dJdf, dJdg = adj.gradients(d, lam)
    dirs = W.random_directions(d.n, 8, seed=1)
    eps = 1e-6
    for dvec in dirs:
        for which, grad in (("f", dJdf), ("g", dJdg)):
            fp, gp, fm, gm = p.f, p.g, p.f, p.g
            if which == "f":
                fp, fm = p.f + eps * dvec, p.f - eps * dvec
            else:
                gp, gm = p.g + eps * dvec, p.g - eps * dvec
            Jp = adj.misfit(d, adj.forward(H, d, fp, gp, k), ut)[0]
            Jm = adj.misfit(d, adj.forward(H, d, fm, gm, k), ut)[0]
            fd = (Jp - Jm) / (2 * eps)
            # exact up to rounding (J is quadratic for a fixed cycle count)
            assert grad @ dvec == pytest.approx(fd, rel=1e-6, abs=50 * 2.2e-16 * abs(J0) / eps)


def test_converged_adjoint_equals_direct(setup32):
    p, d, H = setup32
    ut = W.adjoint_target(d.N)
    u = mg.solve(H, d.rhs(p.f, p.g), tol=1e-12).u
    _, dJdu = adj.misfit(d, u, ut)
    lam = adj.adjoint_solve(H, dJdu, tol=1e-13, max_cycles=80).u
    lam_d = adj.dense_adjoint(d, dJdu)
    assert np.abs(lam - lam_d).max() <= 1e-9 * np.abs(lam_d).max()
    # dJ/dg is supported on the vertices of cut cells only
    _, dJdg = adj.gradients(d, lam)
    cut = mg.cut_vertex_mask((d.cell_type % 4 != 0) & (d.cell_type != 0), d.N)
    assert np.all(dJdg[~cut] == 0.0)
