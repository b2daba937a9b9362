"""Oracle multigrid (test infrastructure): transfers, Galerkin hierarchy,
Gauss-Seidel smoothers, two-grid scheme, V- and W-cycles.

Section 3 of the paper: relaxation (Richardson form, eq. RichRel), the
two-grid correction scheme (Algorithm 1), its recursive V-cycle (gamma* = 1)
and W-cycle (gamma* = 2) and the convergence factor
rho^(m) = ||r^(m)||_inf / ||r^(m-1)||_inf.  Section 5: transfer operators
(two-dimensional shape-function relation, restriction = transpose of
prolongation), Galerkin coarse operators (eq. galerkin, read as R A P with
R = P^T) and extra Gauss-Seidel iterations restricted to cut cells.

Readings (the paper is silent):
* Gauss-Seidel order: four colours c(i,j) = (i mod 2) + 2 (j mod 2) swept
  0, 1, 2, 3 (the paper's lexicographic sweep is also provided).
* Extra smoothing: after every full sweep, eta sweeps over the vertices of
  the cut cells, in the same colour order, on every level but the coarsest.
  A coarse cell is cut when one of its four fine sub-cells is cut.
* Coarsest level: exact solve of the block of nodes with a non-zero diagonal.
* Adjoint (transposed) smoothing: the same phases in reverse order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import geometry as geo


def prolongation(Nc: int) -> sp.csr_matrix:
    """Bilinear prolongation from the (Nc+1)^2 coarse grid to the (2Nc+1)^2
    fine grid: the coefficients of the exact shape-function relation
    phi_2h,k = sum of 1, 1/2, 1/4 times the fine shape functions around the
    fine node (2I, 2J) (section 5.1).  Restriction is its transpose."""
    Nf = 2 * Nc
    rows, cols, vals = [], [], []
    for I in range(Nc + 1):
        for d, w in ((-1, 0.5), (0, 1.0), (1, 0.5)):
            i = 2 * I + d
            if 0 <= i <= Nf:
                rows.append(i)
                cols.append(I)
                vals.append(w)
    P1 = sp.csr_matrix((vals, (rows, cols)), shape=(Nf + 1, Nc + 1))
    return sp.kron(P1, P1, format="csr")  # row (j, i) -> j (Nf+1) + i


def node_colours(N: int) -> np.ndarray:
    i, j = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="xy")
    return ((i % 2) + 2 * (j % 2)).ravel()


def cut_vertex_mask(cell_cut: np.ndarray, N: int) -> np.ndarray:
    """Nodes that are a vertex of at least one cut cell."""
    m = np.zeros((N + 1, N + 1), dtype=bool)
    cc = cell_cut.reshape(N, N)  # [cj, ci]
    m[:-1, :-1] |= cc
    m[:-1, 1:] |= cc
    m[1:, 1:] |= cc
    m[1:, :-1] |= cc
    return m.ravel()


def coarsen_cut_cells(cell_cut: np.ndarray, N: int) -> np.ndarray:
    """A coarse cell is cut iff one of its four fine sub-cells is cut."""
    cc = cell_cut.reshape(N, N)
    return (cc[0::2, 0::2] | cc[0::2, 1::2] | cc[1::2, 0::2] | cc[1::2, 1::2]).ravel()


@dataclass
class Level:
    N: int
    A: sp.csr_matrix
    P: sp.csr_matrix | None          # prolongation from level+1 to this level
    diag: np.ndarray = field(init=False)
    active: np.ndarray = field(init=False)
    cut: np.ndarray | None = None     # bool mask of extra-smoothing nodes
    colour_rows: list = field(default_factory=list)
    colour_A: list = field(default_factory=list)
    cut_rows: list = field(default_factory=list)
    cut_A: list = field(default_factory=list)

    def __post_init__(self):
        self.diag = self.A.diagonal()
        self.active = self.diag != 0.0


@dataclass
class Hierarchy:
    levels: list
    coarse_idx: np.ndarray
    coarse_chol: tuple | None
    coarse_lu: object | None

    @property
    def L(self):
        return len(self.levels) - 1

    def coarse_solve(self, b):
        x = np.zeros_like(b)
        if len(self.coarse_idx) == 0:
            return x
        rhs = b[self.coarse_idx]
        if self.coarse_chol is not None:
            x[self.coarse_idx] = scipy.linalg.cho_solve(self.coarse_chol, rhs)
        else:
            x[self.coarse_idx] = self.coarse_lu.solve(rhs)
        return x


def build_hierarchy(disc, coarsest_n=4, dense_limit=4000, rediscretise=None) -> Hierarchy:
    """Galerkin hierarchy A_{l+1} = P^T A_l P down to a grid of coarsest_n
    cells per side, computed as a generic sparse triple product.

    rediscretise = (psi, kw) instead assembles every coarse operator from
    scratch on its own grid (section 4.3 and section 5, the alternative to the
    Galerkin condition): psi, the unsnapped fine nodal level set, is injected
    at the coarse nodes (coarse node (I, J) is fine node (2I, 2J)) and
    assembled with the fine grid's parameters kw (gamma, alpha, rule,
    lambda_fixed, and a Neumann indicator chi, injected like psi) and the
    coarse cell size; the extra-smoothing set of a coarse level is then the
    vertices of its own cut cells."""
    N = disc.N
    if N % coarsest_n or (N // coarsest_n) & (N // coarsest_n - 1):
        raise ValueError("N must be coarsest_n times a power of two")
    if rediscretise is not None:
        from . import assembly as asm
        psi_in, akw = rediscretise
        psi_in = np.asarray(psi_in, dtype=np.float64).reshape(N + 1, N + 1)
        akw = dict(akw)
        chi_in = akw.pop("chi", None)
        if chi_in is not None:
            chi_in = np.asarray(chi_in, dtype=np.float64).reshape(N + 1, N + 1)
    cell_cut = (disc.cell_type != geo.EXTERNAL) & (disc.cell_type != geo.INTERNAL)
    A = disc.A.tocsr()
    levels = []
    while True:
        P = prolongation(N // 2) if N > coarsest_n else None
        lv = Level(N, A, P)
        col = node_colours(N)
        for c in range(4):
            rows = np.nonzero(lv.active & (col == c))[0]
            lv.colour_rows.append(rows)
            lv.colour_A.append(A[rows])
        if P is not None:
            lv.cut = cut_vertex_mask(cell_cut, N) & lv.active
            for c in range(4):
                rows = np.nonzero(lv.cut & (col == c))[0]
                lv.cut_rows.append(rows)
                lv.cut_A.append(A[rows])
        levels.append(lv)
        if P is None:
            break
        if rediscretise is None:
            A = (P.T @ A @ P).tocsr()
            A.eliminate_zeros()
            cell_cut = coarsen_cut_cells(cell_cut, N)
        else:
            step = disc.N // (N // 2)
            chi_c = None if chi_in is None else chi_in[::step, ::step].ravel()
            dc = asm.assemble(psi_in[::step, ::step].ravel(), N // 2, box=disc.box, chi=chi_c, **akw)
            A = dc.A.tocsr()
            cell_cut = (dc.cell_type != geo.EXTERNAL) & (dc.cell_type != geo.INTERNAL)
        N //= 2
    last = levels[-1]
    idx = np.nonzero(last.active)[0]
    Ab = last.A[idx][:, idx]
    chol = lu = None
    if len(idx) <= dense_limit:
        chol = scipy.linalg.cho_factor(Ab.toarray(), lower=True)
    else:
        lu = spla.splu(Ab.tocsc())
    return Hierarchy(levels, idx, chol, lu)


# ----------------------------------------------------------------------------
# Smoothers
# ----------------------------------------------------------------------------

def _phase(x, b, rows, Arows, diag):
    """One colour phase: x_i += (b_i - (A x)_i) / a_ii for the rows given.
    Rows of one colour are not coupled by the 9-point stencil, so this is
    exactly the Gauss-Seidel update of those nodes."""
    if len(rows):
        x[rows] += (b[rows] - Arows @ x) / diag[rows]


def smoothing_step(lv: Level, x, b, eta, reverse=False):
    """One smoothing step: a full four-colour Gauss-Seidel sweep followed by
    eta sweeps restricted to the cut-cell vertices (section 5.3, extra
    smoothing on cut cells).  reverse=True applies the transposed step
    (every phase in reverse order), used by the adjoint cycle."""
    order = (0, 1, 2, 3)
    if not reverse:
        for c in order:
            _phase(x, b, lv.colour_rows[c], lv.colour_A[c], lv.diag)
        for _ in range(eta):
            for c in order:
                _phase(x, b, lv.cut_rows[c], lv.cut_A[c], lv.diag)
    else:
        for _ in range(eta):
            for c in reversed(order):
                _phase(x, b, lv.cut_rows[c], lv.cut_A[c], lv.diag)
        for c in reversed(order):
            _phase(x, b, lv.colour_rows[c], lv.colour_A[c], lv.diag)


def lexicographic_step(lv: Level, x, b, eta):
    """The paper's Gauss-Seidel, P = lower triangle of A including the
    diagonal (section 4.1), in the node order k = i + j (N+1), followed by eta
    lexicographic sweeps on the cut-cell vertices."""
    a = np.nonzero(lv.active)[0]
    Aa = lv.A[a][:, a].tocsr()
    r = b[a] - Aa @ x[a]
    x[a] += spla.spsolve_triangular(sp.tril(Aa, format="csr"), r, lower=True)
    if eta and lv.cut is not None:
        c = np.nonzero(lv.cut)[0]
        Ac = lv.A[c][:, c].tocsr()
        Lc = sp.tril(Ac, format="csr")
        Arows = lv.A[c]
        for _ in range(eta):
            x[c] += spla.spsolve_triangular(Lc, b[c] - Arows @ x, lower=True)


# ----------------------------------------------------------------------------
# Cycles
# ----------------------------------------------------------------------------

def cycle(hier: Hierarchy, x, b, nu1=2, nu2=1, eta=4, gamma_star=1, level=0,
          reverse=False, smoother="colour"):
    """One multigrid cycle on level `level`, updating x in place.

    Pre-smoothing nu1 steps, residual, restriction R = P^T, gamma_star cycles
    on the next level from a zero guess (an exact solve on the coarsest),
    prolongation and correction, post-smoothing nu2 steps (Algorithm 1 made
    recursive, section 3.2).  The unknowns of a level are its active nodes
    (eq. Vhact): the residual is taken there only, and corrections are only
    added there.  With Galerkin operators the residual vanishes at inactive
    nodes anyway; with rediscretised ones an inactive coarse node can receive
    restricted residual, which is not part of the coarse problem."""
    lv = hier.levels[level]
    if level == hier.L:
        x[:] = hier.coarse_solve(b)
        return x
    step = (lambda xx, bb: smoothing_step(lv, xx, bb, eta, reverse)) if smoother == "colour" \
        else (lambda xx, bb: lexicographic_step(lv, xx, bb, eta))
    for _ in range(nu1):
        step(x, b)
    r = np.where(lv.active, b - lv.A @ x, 0.0)
    bc = lv.P.T @ r
    xc = np.zeros_like(bc)
    for _ in range(gamma_star):
        cycle(hier, xc, bc, nu1, nu2, eta, gamma_star, level + 1, reverse, smoother)
    x += np.where(lv.active, lv.P @ xc, 0.0)
    for _ in range(nu2):
        step(x, b)
    return x


@dataclass
class SolveResult:
    u: np.ndarray
    hist: np.ndarray       # ||F - A u_m||_inf, m = 0..n
    hist_l2: np.ndarray
    cycles: int
    converged: bool

    @property
    def rho(self):
        """rho^(m) = ||r^(m)|| / ||r^(m-1)|| (section 3.1, l-infinity norm)."""
        return self.hist[1:] / self.hist[:-1]


def solve(hier: Hierarchy, F, tol=1e-10, max_cycles=50, u0=None, nu1=2, nu2=1,
          eta=4, gamma_star=1, reverse=False, smoother="colour") -> SolveResult:
    """Repeat cycles from u0 (zero by default) until
    ||F - A u||_inf <= tol ||F||_inf or max_cycles cycles were done."""
    A = hier.levels[0].A
    active = hier.levels[0].active
    u = np.zeros_like(F) if u0 is None else np.where(active, u0, 0.0)
    r = F - A @ u
    hist = [np.abs(r).max()]
    hist2 = [np.linalg.norm(r)]
    fn = np.abs(F).max()
    conv = hist[0] <= tol * fn
    m = 0
    while not conv and m < max_cycles:
        cycle(hier, u, F, nu1, nu2, eta, gamma_star, 0, reverse, smoother)
        m += 1
        r = F - A @ u
        hist.append(np.abs(r).max())
        hist2.append(np.linalg.norm(r))
        conv = hist[-1] <= tol * fn
    return SolveResult(u, np.array(hist), np.array(hist2), m, bool(conv))


def rho_protocol(hier: Hierarchy, iters=30, window=(21, 30), **kw) -> float:
    """The paper's convergence-factor protocol (section 5.3): homogeneous
    problem, u^(0) = 1, `iters` cycles, rho = mean of rho^(m) over the window."""
    n = hier.levels[0].A.shape[0]
    res = solve(hier, np.zeros(n), tol=-1.0, max_cycles=iters, u0=np.ones(n), **kw)
    rho = res.rho
    return float(np.mean(rho[window[0] - 1:window[1]]))


def two_grid(disc, **kw) -> Hierarchy:
    """Two-grid correction scheme (Algorithm 1): one coarse level, solved exactly."""
    return build_hierarchy(disc, coarsest_n=disc.N // 2, **kw)
