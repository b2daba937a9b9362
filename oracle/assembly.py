"""Oracle assembly of the ghost-FEM system (test infrastructure).

Discrete problem (section 2, eqs. disc_bil_form and disc_rhs), summed over the
active cells K after snapping:

    a_h(u, v) = sum_K  int_{K cap Omega} grad u . grad v
                      + int_{K cap Gamma} lambda_K u v - (n . grad u) v - (n . grad v) u
    l_h(v)    = sum_K  int_{K cap Omega} f v
                      + int_{K cap Gamma} lambda_K g v - (n . grad v) g

with lambda_K = gamma C(K) (section 5.2).  On one cell, with phi_i the four
Q1 shape functions and

    S_ij = int_{K cap Omega} grad phi_i . grad phi_j      M_ij = int_{K cap Omega} phi_i phi_j
    B_ij = int_{K cap Gamma} (n . grad phi_j) phi_i       L_ij = int_{K cap Gamma} phi_i phi_j

the element matrix is A_K = S - B - B^T + lambda_K L.  With the global rule
of section 5.2 one lambda = gamma C serves every cut cell, C the largest
eigenvalue of the global pencil (global_eigen_constant).  The data f and g enter
through their nodal Q1 interpolants (a reading: the paper writes exact
integrals of f and g), so that F = M f + G g with G_K = lambda_K L - B^T,
i.e. G_ij = int lambda_K phi_i phi_j - (n . grad phi_i) phi_j.

Mixed boundaries (section 2, Gamma = Gamma_D + Gamma_N).  The penalty and the
two Nitsche terms act on Gamma_D only; Gamma_N contributes the load
int_{K cap Gamma_N} g_N v and nothing to a_h.  Reading: the paper does not say
how a discrete interface segment is assigned to Gamma_D or Gamma_N.  Here the
caller gives a nodal indicator chi; a segment is a Neumann segment when the
bilinear interpolant of chi at the segment's midpoint is > 0, else Dirichlet.
With g_N replaced by its nodal interpolant the load is GN g_N,
GN_ij = int_{K cap Gamma_N} phi_i phi_j.  B, L, the penalty and C(K) use the
Dirichlet segments only; a cell with no Dirichlet segment has lambda_K = 0.

Global matrices live on the full (N+1)^2 node grid (k = i + j (N+1)); rows and
columns of nodes that touch no active cell are empty.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from . import geometry as geo
from .quadrature import polygon_rule, q1_basis, q1_grad, segment_rule


def interior_matrices(h):
    """Exact Q1 stiffness and mass matrices of a full square cell of side h,
    vertices counter-clockwise.  The stiffness is independent of h in 2D."""
    S = np.array([[4.0, -1.0, -2.0, -1.0],
                  [-1.0, 4.0, -1.0, -2.0],
                  [-2.0, -1.0, 4.0, -1.0],
                  [-1.0, -2.0, -1.0, 4.0]]) / 6.0
    M = np.array([[4.0, 2.0, 1.0, 2.0],
                  [2.0, 4.0, 2.0, 1.0],
                  [1.0, 2.0, 4.0, 2.0],
                  [2.0, 1.0, 2.0, 4.0]]) * (h * h / 36.0)
    return S, M


def reference_integrals(polys, segs):
    """Reference-cell integrals (h = 1) over the polygons and segments:
    S, M, B, L as in the module docstring and Kn_ij = int (n.grad phi_i)(n.grad phi_j)."""
    S = np.zeros((4, 4))
    M = np.zeros((4, 4))
    B = np.zeros((4, 4))
    L = np.zeros((4, 4))
    Kn = np.zeros((4, 4))
    for poly in polys:
        pts, w = polygon_rule(poly)
        phi = q1_basis(pts)
        gr = q1_grad(pts)
        S += np.einsum("imk,jmk,m->ij", gr, gr, w)
        M += np.einsum("im,jm,m->ij", phi, phi, w)
    for P, Q in segs:
        d = np.asarray(Q) - np.asarray(P)
        length = float(np.hypot(d[0], d[1]))
        if length == 0.0:
            continue  # degenerate segment: contributes nothing
        n = np.array([d[1], -d[0]]) / length  # outward: right of P -> Q
        pts, w = segment_rule(P, Q)
        phi = q1_basis(pts)
        dn = q1_grad(pts) @ n  # (4, m)
        B += np.einsum("jm,im,m->ij", dn, phi, w)
        L += np.einsum("im,jm,m->ij", phi, phi, w)
        Kn += np.einsum("im,jm,m->ij", dn, dn, w)
    # the symmetric integrals are symmetric in exact arithmetic; remove the
    # rounding-order asymmetry of the sums so that A_K = A_K^T exactly
    sym = lambda X: 0.5 * (X + X.T)  # noqa: E731
    return sym(S), sym(M), B, sym(L), sym(Kn)


def local_eigen_constant(polys, segs):
    """C(K) h from the local generalised eigenproblem of section 5.2:
    Kn v = Lambda S v with Kn the boundary normal-derivative matrix and S the
    cut-cell stiffness.  Both vanish on constants, so the eigenvalue is taken
    in the rank sense of section 4.4 (restriction to the complement of the
    constants) and C = max Lambda."""
    S, _, _, _, Kn = reference_integrals(polys, segs)
    Q = np.linalg.svd(np.ones((1, 4)))[2][1:].T  # 4x3 basis orthogonal to constants
    return float(scipy.linalg.eigh(Q.T @ Kn @ Q, Q.T @ S @ Q, eigvals_only=True).max())


def is_neumann_segment(P, Q, chi4):
    """Segment P -> Q (reference coordinates) is a Neumann segment when the
    bilinear interpolant of the vertex values chi4 at its midpoint is > 0
    (the reading in the module docstring).  The interpolant is summed in the
    vertex order v0..v3."""
    mx = 0.5 * (P[0] + Q[0])
    my = 0.5 * (P[1] + Q[1])
    val = (1.0 - mx) * (1.0 - my) * chi4[0]
    val += mx * (1.0 - my) * chi4[1]
    val += mx * my * chi4[2]
    val += (1.0 - mx) * my * chi4[3]
    return val > 0.0


def split_segments(segs, chi4):
    """(Dirichlet segments, Neumann segments); all Dirichlet when chi4 is None."""
    if chi4 is None:
        return list(segs), []
    dseg, nseg = [], []
    for P, Q in segs:
        (nseg if is_neumann_segment(P, Q, chi4) else dseg).append((P, Q))
    return dseg, nseg


def cut_element(psi4, h, gamma=2.0, rule=geo.STAB_PAPER, lambda_fixed=0.0, chi4=None):
    """Element matrices (A_K, M_K, G_K, GN_K) and (type, C, lambda) of one cut
    cell.  chi4: indicator values at v0..v3 (None: the whole interface is
    Dirichlet)."""
    g = geo.cut_geometry(psi4)
    t, polys, segs, _ = g
    dseg, nseg = split_segments(segs, chi4)
    S, Mr, B, L, _ = reference_integrals(polys, dseg)
    if nseg:
        _, _, _, LN, _ = reference_integrals([], nseg)
    else:
        LN = np.zeros((4, 4))
    if not dseg and segs:
        C = 0.0
        lam = 0.0   # no Dirichlet segment: no penalty
    elif rule == geo.STAB_FIXED:
        C = 0.0
        lam = lambda_fixed
    elif rule == geo.STAB_LOCAL_EIG:
        C = local_eigen_constant(polys, dseg) / h
        lam = gamma * C
    else:
        C = geo.stabilization_constant(psi4, h, rule, geometry=g)
        lam = gamma * C
    lam_ref = lam * h  # lambda_K L_phys = (lambda_K h) L_ref
    A = S - B - B.T + lam_ref * L
    G = lam_ref * L - B.T
    return A, Mr * (h * h), G, LN * h, (t, C, lam)


@dataclass
class Discretisation:
    N: int
    h: float
    box: tuple
    psi: np.ndarray        # snapped nodal level set
    cell_type: np.ndarray  # (N*N,) type codes of geometry
    cell_lambda: np.ndarray
    cell_C: np.ndarray
    A: sp.csr_matrix
    M: sp.csr_matrix
    G: sp.csr_matrix
    active: np.ndarray     # (n,) bool: vertex of an active cell
    GN: sp.csr_matrix | None = None  # Neumann load matrix (None: no Neumann segment)

    @property
    def n(self):
        return (self.N + 1) ** 2

    def rhs(self, f, g, gN=None):
        """F = M f + G g (+ GN g_N): nodal interpolants of f, g_D and g_N."""
        F = self.M @ f + self.G @ g
        if gN is not None and self.GN is not None:
            F = F + self.GN @ gN
        return F

    @property
    def cut_cells(self):
        t = self.cell_type
        return np.nonzero((t != geo.EXTERNAL) & (t != geo.INTERNAL))[0]


def global_pencil(psi4, ctype, N, h, chi4=None):
    """The matrices of the global generalised eigenproblem of section 5.2 on
    the full node grid: K_ij = int_{Gamma_D} (n.grad phi_i)(n.grad phi_j)
    (physical K = K_ref / h) and S_ij = int_Omega grad phi_i . grad phi_j,
    with the boolean mask of the active nodes."""
    V = cell_vertex_indices(N)
    n = (N + 1) ** 2
    S_int, _ = interior_matrices(h)
    rows, cols, sval, kval = [], [], [], []
    inner = np.nonzero(ctype == geo.INTERNAL)[0]
    Vi = V[inner]
    rows.append(np.repeat(Vi[:, :, None], 4, axis=2).ravel())
    cols.append(np.repeat(Vi[:, None, :], 4, axis=1).ravel())
    sval.append(np.broadcast_to(S_int, (len(inner), 4, 4)).ravel())
    kval.append(np.zeros(len(inner) * 16))
    for c in np.nonzero((ctype != geo.EXTERNAL) & (ctype != geo.INTERNAL))[0]:
        _, polys, segs, _ = geo.cut_geometry(psi4[c])
        dseg, _ = split_segments(segs, None if chi4 is None else chi4[c])
        S, _, _, _, Kn = reference_integrals(polys, dseg)
        v = V[c]
        rows.append(np.repeat(v, 4))
        cols.append(np.tile(v, 4))
        sval.append(S.ravel())
        kval.append((Kn / h).ravel())
    r = np.concatenate(rows)
    c_ = np.concatenate(cols)
    S = sp.coo_matrix((np.concatenate(sval), (r, c_)), shape=(n, n)).tocsr()
    K = sp.coo_matrix((np.concatenate(kval), (r, c_)), shape=(n, n)).tocsr()
    act = np.zeros(n, dtype=bool)
    act[V[ctype != geo.EXTERNAL].ravel()] = True
    return K, S, act


def global_eigen_constant(psi4, ctype, N, h, chi4=None):
    """C of the global generalised eigenproblem of section 5.2: the largest
    Lambda with K v = Lambda S v over the active nodes (global_pencil).

    Both matrices vanish on the constants, and the Rayleigh quotient
    v^T K v / v^T S v does not change when a constant is added to v, so the
    eigenvalues are taken on the complement of the constants (the rank sense
    of section 4.4) by fixing v = 0 at one active node; for a connected active
    domain S is then positive definite."""
    K, S, act = global_pencil(psi4, ctype, N, h, chi4)
    idx = np.nonzero(act)[0][1:]  # fix v = 0 at the first active node
    S = S[idx][:, idx]
    K = K[idx][:, idx]
    S = 0.5 * (S + S.T)
    K = 0.5 * (K + K.T)
    if len(idx) <= 4000:
        return float(scipy.linalg.eigh(K.toarray(), S.toarray(), eigvals_only=True).max())
    import scipy.sparse.linalg as spla
    return float(spla.eigsh(K.tocsc(), k=1, M=S.tocsc(), which="LA", tol=1e-14,
                            return_eigenvectors=False)[0])


def cell_vertex_indices(N):
    """(N*N, 4) global node indices of v0..v3 of every cell."""
    ci, cj = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    k0 = (ci + cj * (N + 1)).ravel()
    return np.stack([k0, k0 + 1, k0 + N + 2, k0 + N + 1], axis=1)


def assemble(psi, N, box=(-1.0, -1.0, 1.0, 1.0), gamma=2.0, alpha=1.75,
             rule=geo.STAB_PAPER, lambda_fixed=0.0, snap=True, chi=None):
    """Snap, classify and assemble A, M, G (and GN when chi, the nodal
    Neumann indicator, is given) on the full node grid."""
    h = (box[2] - box[0]) / N
    psi_s = geo.snap(psi, h, alpha) if snap else np.asarray(psi, dtype=np.float64).copy()
    psi4 = geo.cell_vertex_values(psi_s, N)
    ctype = geo.classify(psi4)
    V = cell_vertex_indices(N)
    n = (N + 1) ** 2

    chi4 = None if chi is None else geo.cell_vertex_values(np.asarray(chi, dtype=np.float64), N)
    C_global = None
    if rule == geo.STAB_GLOBAL:
        # one lambda = gamma C for every cut cell (section 5.2)
        C_global = global_eigen_constant(psi4, ctype, N, h, chi4)
        rule, lambda_fixed = geo.STAB_FIXED, gamma * C_global
    rows, cols, aval, mval, gval, nval = [], [], [], [], [], []
    S_int, M_int = interior_matrices(h)
    inner = np.nonzero(ctype == geo.INTERNAL)[0]
    if len(inner):
        Vi = V[inner]
        rows.append(np.repeat(Vi[:, :, None], 4, axis=2).ravel())
        cols.append(np.repeat(Vi[:, None, :], 4, axis=1).ravel())
        aval.append(np.broadcast_to(S_int, (len(inner), 4, 4)).ravel())
        mval.append(np.broadcast_to(M_int, (len(inner), 4, 4)).ravel())
        gval.append(np.zeros(len(inner) * 16))
        nval.append(np.zeros(len(inner) * 16))

    cell_lambda = np.zeros(N * N)
    cell_C = np.zeros(N * N)
    cut = np.nonzero((ctype != geo.EXTERNAL) & (ctype != geo.INTERNAL))[0]
    for c in cut:
        A_K, M_K, G_K, N_K, (_, C, lam) = cut_element(
            psi4[c], h, gamma, rule, lambda_fixed, None if chi4 is None else chi4[c])
        cell_lambda[c] = lam
        cell_C[c] = C if C_global is None else C_global
        v = V[c]
        rows.append(np.repeat(v, 4))
        cols.append(np.tile(v, 4))
        aval.append(A_K.ravel())
        mval.append(M_K.ravel())
        gval.append(G_K.ravel())
        nval.append(N_K.ravel())

    if rows:
        r = np.concatenate(rows)
        c_ = np.concatenate(cols)
        A = sp.coo_matrix((np.concatenate(aval), (r, c_)), shape=(n, n)).tocsr()
        M = sp.coo_matrix((np.concatenate(mval), (r, c_)), shape=(n, n)).tocsr()
        G = sp.coo_matrix((np.concatenate(gval), (r, c_)), shape=(n, n)).tocsr()
        GN = sp.coo_matrix((np.concatenate(nval), (r, c_)), shape=(n, n)).tocsr()
        GN = ((GN + GN.T) * 0.5).tocsr()
        # A and M are symmetric in exact arithmetic; make them so in floating
        # point too (the duplicate summation order may differ between (i,j)
        # and (j,i))
        A = ((A + A.T) * 0.5).tocsr()
        M = ((M + M.T) * 0.5).tocsr()
    else:
        A = M = G = GN = sp.csr_matrix((n, n))
    active = np.zeros(n, dtype=bool)
    active[V[ctype != geo.EXTERNAL].ravel()] = True
    return Discretisation(N, h, tuple(box), psi_s, ctype, cell_lambda, cell_C,
                          A, M, G, active, GN if chi is not None else None)
