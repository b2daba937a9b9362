// Setup on the device, part 1: snapping back to grid, cut-cell geometry,
// the stabilisation constant C(K), and the fine-grid stencils of A, M and G.
//
// Geometry (section 2; section 5.2 "Global and local stabilization
// parameters"): psi < 0 is inside, psi = 0 (including snapped nodes) counts as
// outside; a cell's piece K cap Omega is the polygon of its inside vertices and
// the points where psi, linearly interpolated along an edge, vanishes.  The
// interface K cap Gamma is the straight segment(s) joining those points.
// Element integrals (eqs. disc_bil_form / disc_rhs) are exact: a degree-5
// seven-point triangle rule over a fan of triangles from the polygon's vertex
// mean, and four-point Gauss-Lobatto on the segments (degree 5), which covers
// the degree-4 mass and penalty integrands.
//
// Mixed boundaries (section 2): given a nodal indicator chi, a segment whose
// midpoint has a positive bilinear interpolant of chi belongs to Gamma_N (the
// paper leaves the assignment of discrete segments open; this is the rule the
// library uses).  Penalty, Nitsche terms and C(K) use the Dirichlet segments
// only; the Neumann segments give the boundary mass GN of the load
// int_{Gamma_N} g_N v; a cell with no Dirichlet segment has lambda_K = 0.
#include <cmath>

#include "mgfem_internal.h"

namespace mgfem {
namespace {

struct P2 {
  double x, y;
};

// --- Q1 basis on the reference cell, vertices counter-clockwise from (0,0)
__host__ __device__ inline void q1_val(double x, double y, double v[4]) {
  v[0] = (1.0 - x) * (1.0 - y);
  v[1] = x * (1.0 - y);
  v[2] = x * y;
  v[3] = (1.0 - x) * y;
}
__host__ __device__ inline void q1_grad(double x, double y, double gx[4], double gy[4]) {
  gx[0] = -(1.0 - y);
  gx[1] = 1.0 - y;
  gx[2] = y;
  gx[3] = -y;
  gy[0] = -(1.0 - x);
  gy[1] = -x;
  gy[2] = x;
  gy[3] = 1.0 - x;
}

__host__ __device__ inline P2 ref_vertex(int m) {
  return P2{(m == 1 || m == 2) ? 1.0 : 0.0, (m >= 2) ? 1.0 : 0.0};
}

// Cut geometry of one cell in reference coordinates.
struct CutCell {
  int type;
  int npoly;
  int nv[2];
  P2 poly[2][6];
  int nseg;
  P2 sp[2], sq[2];   // segment endpoints; the piece lies to the left of sp -> sq
  int neu[2];        // 1: the segment lies on the Neumann part of the boundary
  double theta[4];   // cut fraction of edge e from its inside end, or -1
};

__host__ __device__ int classify4(const double ps[4]) {
  int in0 = ps[0] < 0.0, in1 = ps[1] < 0.0, in2 = ps[2] < 0.0, in3 = ps[3] < 0.0;
  int k = in0 + in1 + in2 + in3;
  if (k == 0) return kExternal;
  if (k == 4) return kInternal;
  if (k == 1) return kTriangle;
  if (k == 3) return kPentagon;
  if (in0 == in2) {  // two diagonal inside vertices: saddle
    double mean = 0.25 * (ps[0] + ps[1] + ps[2] + ps[3]);
    return mean < 0.0 ? kSaddleHex : kSaddleSplit;
  }
  return kQuad;
}

__host__ __device__ void cut_cell(const double ps[4], CutCell& cc) {
  cc.type = classify4(ps);
  cc.npoly = 0;
  cc.nseg = 0;
  cc.neu[0] = cc.neu[1] = 0;
  P2 cp[4];
  bool in[4];
  for (int m = 0; m < 4; ++m) in[m] = ps[m] < 0.0;
  for (int e = 0; e < 4; ++e) {
    int a = e, b = (e + 1) & 3;
    cc.theta[e] = -1.0;
    if (in[a] != in[b]) {
      int pin = in[a] ? a : b, pout = in[a] ? b : a;
      double t = ps[pin] / (ps[pin] - ps[pout]);
      cc.theta[e] = t;
      P2 vi = ref_vertex(pin), vo = ref_vertex(pout);
      cp[e] = P2{vi.x + t * (vo.x - vi.x), vi.y + t * (vo.y - vi.y)};
    }
  }
  if (cc.type == kExternal) return;
  if (cc.type == kInternal) {
    cc.npoly = 1;
    cc.nv[0] = 4;
    for (int m = 0; m < 4; ++m) cc.poly[0][m] = ref_vertex(m);
    return;
  }
  if (cc.type == kSaddleSplit) {
    for (int p = 0; p < 4; ++p) {
      if (!in[p]) continue;
      int q = cc.npoly++;
      int eprev = (p + 3) & 3;
      cc.nv[q] = 3;
      cc.poly[q][0] = ref_vertex(p);
      cc.poly[q][1] = cp[p];
      cc.poly[q][2] = cp[eprev];
      cc.sp[cc.nseg] = cp[p];
      cc.sq[cc.nseg] = cp[eprev];
      ++cc.nseg;
    }
    return;
  }
  // one connected piece: walk the cell boundary counter-clockwise
  cc.npoly = 1;
  int nv = 0;
  int exits[2], entries[2], nex = 0, nen = 0;
  int order[4];  // walk position of each cut edge's point
  for (int e = 0; e < 4; ++e) {
    if (in[e]) cc.poly[0][nv++] = ref_vertex(e);
    if (cc.theta[e] >= 0.0) {
      order[e] = nv;
      cc.poly[0][nv++] = cp[e];
      if (in[e]) exits[nex++] = e;
      else entries[nen++] = e;
    }
  }
  cc.nv[0] = nv;
  // pair each exit with the next entry along the walk (cyclically)
  for (int a = 0; a < nex; ++a) {
    int best = -1, bestd = 99;
    for (int b = 0; b < nen; ++b) {
      int d = (order[entries[b]] - order[exits[a]] + nv) % nv;
      if (d < bestd) {
        bestd = d;
        best = entries[b];
      }
    }
    cc.sp[cc.nseg] = cp[exits[a]];
    cc.sq[cc.nseg] = cp[best];
    ++cc.nseg;
  }
}

// Mark the Neumann segments: bilinear interpolant of the vertex values chi at
// the segment midpoint > 0, summed in vertex order without contraction so that
// the decision is the one a plain float64 evaluation takes.
__host__ __device__ void mark_neumann(CutCell& cc, const double chi[4]) {
#pragma clang fp contract(off)
  for (int s = 0; s < cc.nseg; ++s) {
    const double mx = 0.5 * (cc.sp[s].x + cc.sq[s].x), my = 0.5 * (cc.sp[s].y + cc.sq[s].y);
    double v = (1.0 - mx) * (1.0 - my) * chi[0];
    v += mx * (1.0 - my) * chi[1];
    v += mx * my * chi[2];
    v += (1.0 - mx) * my * chi[3];
    cc.neu[s] = v > 0.0 ? 1 : 0;
  }
}

// the cell has segments and every one of them is a Neumann segment
__host__ __device__ inline bool all_neumann(const CutCell& cc) {
  for (int s = 0; s < cc.nseg; ++s)
    if (!cc.neu[s]) return false;
  return cc.nseg > 0;
}

// C(K) h for a triangle with cut sides t1 h, t2 h (eq. c_triangle).
__host__ __device__ double chat_triangle(double t1, double t2) {
  double s2 = t1 * t1 + t2 * t2;
  double t14 = t1 * t1 * t1 * t1, t24 = t2 * t2 * t2 * t2;
  double root = sqrt(3.0 * (t14 * t14 + 10.0 * t14 * t24 + t24 * t24));
  return sqrt(s2) * (3.0 * t14 + 3.0 * t24 + root) / (t1 * t2 * s2 * s2);
}

// C(K) h for a quadrilateral with cut sides t1 h, t2 h (section 5.2); the
// polynomials are evaluated in powers of t2 with coefficients in t1.
__host__ __device__ double chat_quad(double a, double b) {
  double a2 = a * a, b2 = b * b;
  double L = sqrt(1.0 + a2 - 2.0 * a * b + b2);
  double a3 = a2 * a, a4 = a2 * a2, a5 = a4 * a, a6 = a3 * a3, a7 = a6 * a;
  double b3 = b2 * b, b4 = b2 * b2, b5 = b4 * b, b6 = b3 * b3;
  double Q = a6 + 2.0 * a3 * b + b2 - a4 * b2 + b6 + 2.0 * a * (b + b3) -
             a2 * (-1.0 + 2.0 * b2 + b4);
  // P as a polynomial in b: coefficients c[k] of b^k
  double a8 = a4 * a4, a9 = a8 * a, a10 = a5 * a5, a11 = a10 * a, a12 = a6 * a6,
         a13 = a12 * a, a14 = a7 * a7;
  double c[15];
  c[0] = a14 + a12 + 10.0 * a10 + 10.0 * a8 + a6 + a4;
  c[1] = 2.0 * a13 + 16.0 * a11 + 12.0 * a9 + 32.0 * a7 + 10.0 * a5;
  c[2] = -5.0 * a12 - 22.0 * a10 - 38.0 * a8 - 32.0 * a6 - a4 - 2.0 * a2;
  c[3] = -28.0 * a11 - 40.0 * a9 - 32.0 * a7 - 56.0 * a5 - 20.0 * a3;
  c[4] = 73.0 * a10 + 63.0 * a8 + 136.0 * a6 + 104.0 * a4 - a2 + 1.0;
  c[5] = -34.0 * a9 + 24.0 * a7 - 176.0 * a5 - 56.0 * a3 + 10.0 * a;
  c[6] = -69.0 * a8 - 84.0 * a6 + 136.0 * a4 - 32.0 * a2 + 1.0;
  c[7] = 120.0 * a7 + 24.0 * a5 - 32.0 * a3 + 32.0 * a;
  c[8] = -69.0 * a6 + 63.0 * a4 - 38.0 * a2 + 10.0;
  c[9] = -34.0 * a5 - 40.0 * a3 + 12.0 * a;
  c[10] = 73.0 * a4 - 22.0 * a2 + 10.0;
  c[11] = -28.0 * a3 + 16.0 * a;
  c[12] = -5.0 * a2 + 1.0;
  c[13] = 2.0 * a;
  c[14] = 1.0;
  double P = c[14];
  for (int k = 13; k >= 0; --k) P = P * b + c[k];
  double D = a7 + a6 * b + a5 * (2.0 - 3.0 * b2) + a3 * (b2 - 1.0) * (b2 - 1.0) +
             b3 * (1.0 + b2) * (1.0 + b2) + a4 * b * (6.0 + b2) + a * b2 * (5.0 + 6.0 * b2 + b4) +
             a2 * (5.0 * b - 2.0 * b3 - 3.0 * b5);
  return (3.0 * L * Q + sqrt(3.0 * P)) / D;
}

// Radon's seven-point degree-5 rule: barycentric points and weights
__host__ __device__ inline void radon(int q, double& l1, double& l2, double& l3, double& w) {
  const double s15 = 3.872983346207417;  // sqrt(15)
  const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
  const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
  if (q == 0) {
    l1 = l2 = l3 = 1.0 / 3.0;
    w = 9.0 / 40.0;
    return;
  }
  double a = q <= 3 ? a1 : a2;
  double b = 1.0 - 2.0 * a;
  w = q <= 3 ? w1 : w2;
  int r = (q - 1) % 3;
  l1 = r == 0 ? b : a;
  l2 = r == 1 ? b : a;
  l3 = r == 2 ? b : a;
}

// Full 4x4 reference integrals of a cut cell (h = 1); L, B, Kn over the
// Dirichlet segments, LN (boundary mass) over the Neumann segments.
struct CellInt {
  double S[4][4], Mm[4][4], L[4][4], B[4][4], Kn[4][4], LN[4][4];
};

__host__ __device__ void cell_integrals(const CutCell& cc, CellInt& I) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) I.S[i][j] = I.Mm[i][j] = I.L[i][j] = I.B[i][j] = I.Kn[i][j] = I.LN[i][j] = 0.0;
  for (int q = 0; q < cc.npoly; ++q) {
    int nv = cc.nv[q];
    P2 cen{0.0, 0.0};
    for (int v = 0; v < nv; ++v) {
      cen.x += cc.poly[q][v].x;
      cen.y += cc.poly[q][v].y;
    }
    cen.x /= nv;
    cen.y /= nv;
    for (int v = 0; v < nv; ++v) {
      P2 a = cen, b = cc.poly[q][v], c2 = cc.poly[q][(v + 1) % nv];
      double area = 0.5 * fabs((b.x - a.x) * (c2.y - a.y) - (b.y - a.y) * (c2.x - a.x));
      for (int k = 0; k < 7; ++k) {
        double l1, l2, l3, w;
        radon(k, l1, l2, l3, w);
        double x = l1 * a.x + l2 * b.x + l3 * c2.x;
        double y = l1 * a.y + l2 * b.y + l3 * c2.y;
        double ph[4], gx[4], gy[4];
        q1_val(x, y, ph);
        q1_grad(x, y, gx, gy);
        double wa = w * area;
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) {
            I.S[i][j] += wa * (gx[i] * gx[j] + gy[i] * gy[j]);
            I.Mm[i][j] += wa * (ph[i] * ph[j]);
          }
      }
    }
  }
  // four-point Gauss-Lobatto on [0, 1]
  const double r5 = 0.4472135954999579;  // 1/sqrt(5)
  const double gt[4] = {0.0, 0.5 * (1.0 - r5), 0.5 * (1.0 + r5), 1.0};
  const double gw[4] = {1.0 / 12.0, 5.0 / 12.0, 5.0 / 12.0, 1.0 / 12.0};
  for (int sgi = 0; sgi < cc.nseg; ++sgi) {
    P2 P = cc.sp[sgi], Q = cc.sq[sgi];
    double dx = Q.x - P.x, dy = Q.y - P.y;
    double len = sqrt(dx * dx + dy * dy);
    if (len == 0.0) continue;
    double nx = dy / len, ny = -dx / len;  // outward: to the right of P -> Q
    if (cc.neu[sgi]) {
      for (int k = 0; k < 4; ++k) {
        double ph[4];
        q1_val(P.x + gt[k] * dx, P.y + gt[k] * dy, ph);
        double wl = gw[k] * len;
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) I.LN[i][j] += wl * (ph[i] * ph[j]);
      }
      continue;
    }
    for (int k = 0; k < 4; ++k) {
      double x = P.x + gt[k] * dx, y = P.y + gt[k] * dy;
      double ph[4], gx[4], gy[4], dn[4];
      q1_val(x, y, ph);
      q1_grad(x, y, gx, gy);
      for (int i = 0; i < 4; ++i) dn[i] = nx * gx[i] + ny * gy[i];
      double wl = gw[k] * len;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          I.L[i][j] += wl * (ph[i] * ph[j]);
          I.B[i][j] += wl * (dn[j] * ph[i]);  // int (n . grad phi_j) phi_i
          I.Kn[i][j] += wl * (dn[i] * dn[j]);
        }
    }
  }
}

// Largest eigenvalue of the symmetric 3x3 matrix m (closed-form trigonometric solution).
__host__ __device__ double sym3_max_eig(const double m[3][3]) {
  double p1 = m[0][1] * m[0][1] + m[0][2] * m[0][2] + m[1][2] * m[1][2];
  double q = (m[0][0] + m[1][1] + m[2][2]) / 3.0;
  double p2 = (m[0][0] - q) * (m[0][0] - q) + (m[1][1] - q) * (m[1][1] - q) +
              (m[2][2] - q) * (m[2][2] - q) + 2.0 * p1;
  double p = sqrt(p2 / 6.0);
  if (p == 0.0) return q;
  double bm[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) bm[i][j] = (m[i][j] - (i == j ? q : 0.0)) / p;
  double det = bm[0][0] * (bm[1][1] * bm[2][2] - bm[1][2] * bm[2][1]) -
               bm[0][1] * (bm[1][0] * bm[2][2] - bm[1][2] * bm[2][0]) +
               bm[0][2] * (bm[1][0] * bm[2][1] - bm[1][1] * bm[2][0]);
  double r = fmin(1.0, fmax(-1.0, 0.5 * det));
  return q + 2.0 * p * cos(acos(r) / 3.0);
}

// C(K) h from the local generalised eigenproblem Kn v = Lambda S v on the
// complement of the constants (section 5.2; rank definition of section 4.4).
__host__ __device__ double chat_local_eig(const CellInt& I) {
  // orthonormal basis of the complement of (1,1,1,1)
  const double Qb[3][4] = {{0.5, -0.5, 0.5, -0.5}, {0.5, 0.5, -0.5, -0.5}, {0.5, -0.5, -0.5, 0.5}};
  double s[3][3], k[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double ss = 0.0, kk = 0.0;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          double sym = 0.5 * (I.S[i][j] + I.S[j][i]);
          double kns = 0.5 * (I.Kn[i][j] + I.Kn[j][i]);
          ss += Qb[a][i] * sym * Qb[b][j];
          kk += Qb[a][i] * kns * Qb[b][j];
        }
      s[a][b] = ss;
      k[a][b] = kk;
    }
  // Cholesky s = R R^T, then C = R^{-1} k R^{-T}
  double R[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j <= i; ++j) {
      double acc = s[i][j];
      for (int t = 0; t < j; ++t) acc -= R[i][t] * R[j][t];
      R[i][j] = (i == j) ? sqrt(fmax(acc, 1e-300)) : acc / R[j][j];
    }
  double Y[3][3];  // Y = R^{-1} k
  for (int col = 0; col < 3; ++col)
    for (int i = 0; i < 3; ++i) {
      double acc = k[i][col];
      for (int t = 0; t < i; ++t) acc -= R[i][t] * Y[t][col];
      Y[i][col] = acc / R[i][i];
    }
  double Cm[3][3];  // C = Y R^{-T}: solve R Z^T = Y^T row-wise
  for (int row = 0; row < 3; ++row)
    for (int i = 0; i < 3; ++i) {
      double acc = Y[row][i];
      for (int t = 0; t < i; ++t) acc -= R[i][t] * Cm[row][t];
      Cm[row][i] = acc / R[i][i];
    }
  double Cs[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Cs[i][j] = 0.5 * (Cm[i][j] + Cm[j][i]);
  return sym3_max_eig(Cs);
}

// lambda_K h of a cut cell for the given rule (section 5.2).  Triangles use
// the two cut fractions at their inside vertex, quadrilaterals the fraction on
// each cut edge (each from its own inside vertex), pentagons 3 sqrt(2).  A
// saddle split into two triangles takes the larger triangle value, a saddle
// joined into a hexagon the pentagon value.
__host__ __device__ double lambda_h_rule(const double ps[4], const double theta[4], int type,
                                         int rule, double gamma, double lambda_fixed, double h,
                                         double chat_eig) {
  if (rule == MGFEM_STAB_FIXED) return lambda_fixed * h;
  double chat = 0.0;
  if (rule == MGFEM_STAB_LOCAL_EIG) {
    chat = chat_eig;
  } else if (type == kTriangle || type == kSaddleSplit) {
    for (int pv = 0; pv < 4; ++pv)
      if (ps[pv] < 0.0) chat = fmax(chat, chat_triangle(theta[pv], theta[(pv + 3) & 3]));
  } else if (type == kQuad) {
    double a = -1.0, b = -1.0;
    for (int e = 0; e < 4; ++e)
      if (theta[e] >= 0.0) {
        if (a < 0.0) a = theta[e];
        else b = theta[e];
      }
    chat = chat_quad(a, b);
  } else {
    chat = 4.242640687119285;  // 3 sqrt(2), eq. c_pentagon
  }
  return gamma * chat;  // lambda_K h = gamma C(K) h
}

__global__ void k_snap(const double* __restrict__ psi_in, double* __restrict__ psi, int64_t n,
                       double thr, Stats* st) {
  __shared__ unsigned int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) {
    double v = psi_in[k];
    if (v < 0.0 && -v < thr) {
      v = 0.0;
      atomicAdd(&cnt, 1u);
    }
    psi[k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0 && cnt) atomicAdd(&st->snapped, (unsigned long long)cnt);
}

__device__ inline void load_cell_psi(const double* psi, int stride, int ci, int cj, double ps[4]) {
  int64_t k0 = ci + (int64_t)cj * stride;
  ps[0] = psi[k0];
  ps[1] = psi[k0 + 1];
  ps[2] = psi[k0 + stride + 1];
  ps[3] = psi[k0 + stride];
}

__global__ void k_classify(const double* __restrict__ psi, const double* __restrict__ chi, int N,
                           mgfem_params p, double h, uint8_t* __restrict__ ctype, double* __restrict__ clam,
                           uint8_t* __restrict__ cellcut, Stats* st) {
  __shared__ unsigned int cnt[7], ndir;
  __shared__ unsigned long long mint, maxl;
  if (threadIdx.x < 7) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    mint = 0x7ff0000000000000ull;
    maxl = 0;
    ndir = 0;
  }
  __syncthreads();
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t nc = (int64_t)N * N;
  if (c < nc) {
    int ci = (int)(c % N), cj = (int)(c / N);
    double ps[4];
    load_cell_psi(psi, N + 1, ci, cj, ps);
    int t = classify4(ps);
    double lam = 0.0;
    if (t != kExternal && t != kInternal) {
      CutCell cc;
      cut_cell(ps, cc);
      if (chi) {
        double cs[4];
        load_cell_psi(chi, N + 1, ci, cj, cs);
        mark_neumann(cc, cs);
      }
      double chat_eig = 0.0;
      if (p.stab_rule == MGFEM_STAB_LOCAL_EIG) {
        CellInt I;
        cell_integrals(cc, I);
        chat_eig = chat_local_eig(I);
      }
      double lh = lambda_h_rule(ps, cc.theta, t, p.stab_rule, p.gamma, p.lambda_fixed, h, chat_eig);
      lam = all_neumann(cc) ? 0.0 : lh / h;
      if (!all_neumann(cc)) atomicAdd(&ndir, 1u);
      double tmin = 2.0;
      for (int e = 0; e < 4; ++e)
        if (cc.theta[e] >= 0.0) tmin = fmin(tmin, cc.theta[e]);
      atomicMin(&mint, (unsigned long long)__double_as_longlong(tmin));
      atomicMax(&maxl, (unsigned long long)__double_as_longlong(lam));
    }
    ctype[c] = (uint8_t)t;
    clam[c] = lam;
    cellcut[c] = (t != kExternal && t != kInternal) ? 1 : 0;
    atomicAdd(&cnt[t], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 7 && cnt[threadIdx.x])
    atomicAdd(&st->counts[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
  if (threadIdx.x == 0 && ndir) atomicAdd(&st->dirichlet_cells, (unsigned long long)ndir);
  if (threadIdx.x == 0) {
    if (mint != 0x7ff0000000000000ull) atomicMin(&st->min_theta_bits, mint);
    if (maxl) atomicMax(&st->max_lambda_bits, maxl);
  }
}

// local vertex offsets: v0 (0,0), v1 (1,0), v2 (1,1), v3 (0,1)
__constant__ int kVx[4] = {0, 1, 1, 0};
__constant__ int kVy[4] = {0, 0, 1, 1};

// Gather the rows of A, M, G of every node from its (up to) four cells.
// With stiffness_only (the operator of the global eigenproblem) A receives the
// cut stiffness S alone, its stored rows with the diagonal scaled by
// 1 + diag_shift, and Kp the boundary normal-derivative matrix K = Kn / h.
__global__ void k_assemble(const double* __restrict__ psi, const double* __restrict__ chi, int N,
                           mgfem_params p, double h, const uint8_t* __restrict__ ctype,
                           const double* __restrict__ clam, double* __restrict__ A, double* __restrict__ Mm,
                           double* __restrict__ G, double* __restrict__ GN, uint8_t* __restrict__ flags,
                           Stats* st, int stiffness_only, double diag_shift, double* __restrict__ Kp) {
  __shared__ unsigned int nact;
  if (threadIdx.x == 0) nact = 0;
  __syncthreads();
  const int stride = N + 1;
  const int64_t n = (int64_t)stride * stride;
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) {
    int i = (int)(k % stride), j = (int)(k / stride);
    double a[9], m[9], g[9], gn[9], kn[9];
    for (int q = 0; q < 9; ++q) a[q] = m[q] = g[q] = gn[q] = kn[q] = 0.0;
    bool active = false, regular = true;
    // cells around the node, with the node's local vertex number in each
    const int cdx[4] = {-1, 0, 0, -1}, cdy[4] = {-1, -1, 0, 0}, loc[4] = {2, 3, 0, 1};
    const double hh36 = h * h / 36.0;
    for (int s = 0; s < 4; ++s) {
      int ci = i + cdx[s], cj = j + cdy[s];
      if (ci < 0 || cj < 0 || ci >= N || cj >= N) {
        regular = false;
        continue;
      }
      int64_t c = ci + (int64_t)cj * N;
      int t = ctype[c];
      int lv = loc[s];
      if (t != kInternal) regular = false;
      if (t == kExternal) continue;
      active = true;
      if (t == kInternal) {
        for (int mm = 0; mm < 4; ++mm) {
          int dxo = ci + kVx[mm] - i, dyo = cj + kVy[mm] - j;
          int pl = (dxo + 1) + 3 * (dyo + 1);
          int sep = (mm - lv) & 3;  // 0 same, 1/3 edge, 2 opposite
          a[pl] += sep == 0 ? (4.0 / 6.0) : (sep == 2 ? (-2.0 / 6.0) : (-1.0 / 6.0));
          m[pl] += hh36 * (sep == 0 ? 4.0 : (sep == 2 ? 1.0 : 2.0));
        }
      } else {
        double ps[4];
        load_cell_psi(psi, stride, ci, cj, ps);
        CutCell cc;
        cut_cell(ps, cc);
        if (chi) {
          double cs[4];
          load_cell_psi(chi, stride, ci, cj, cs);
          mark_neumann(cc, cs);
        }
        CellInt I;
        cell_integrals(cc, I);
        double lh = clam[c] * h;  // lambda_K h
        for (int mm = 0; mm < 4; ++mm) {
          int dxo = ci + kVx[mm] - i, dyo = cj + kVy[mm] - j;
          int pl = (dxo + 1) + 3 * (dyo + 1);
          // A_K = S - B - B^T + lambda L with the symmetric pair summed first
          if (stiffness_only) {
            a[pl] += I.S[lv][mm];
            kn[pl] += I.Kn[lv][mm] / h;
          } else {
            double sl = I.S[lv][mm] + lh * I.L[lv][mm];
            double nit = I.B[lv][mm] + I.B[mm][lv];
            a[pl] += sl - nit;
          }
          m[pl] += (h * h) * I.Mm[lv][mm];
          // G_ij = lambda L_ij - int (n . grad phi_i) phi_j
          g[pl] += lh * I.L[lv][mm] - I.B[mm][lv];
          gn[pl] += h * I.LN[lv][mm];  // int_{Gamma_N} phi_i phi_j
        }
      }
    }
    if (stiffness_only && active && !regular) a[4] *= 1.0 + diag_shift;
    for (int q = 0; q < 9; ++q) {
      A[q * n + k] = a[q];
      if (Kp) Kp[q * n + k] = kn[q];
      if (Mm) Mm[q * n + k] = m[q];  // mass and boundary load: finest level only
      if (G) G[q * n + k] = g[q];
      if (GN) GN[q * n + k] = gn[q];
    }
    uint8_t f = 0;
    if (active) f |= kFlagActive;
    if (active && !regular) f |= kFlagStored;
    flags[k] = f;
    if (active) atomicAdd(&nact, 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0 && nact) atomicAdd(&st->active, (unsigned long long)nact);
}

// psi of a coarse grid: the fine input at every step-th node in each direction
__global__ void k_inject(const double* __restrict__ psi_in, int N0, int step, double* __restrict__ out, int Nl) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nl = (int64_t)(Nl + 1) * (Nl + 1);
  if (k >= nl) return;
  const int I = (int)(k % (Nl + 1)), J = (int)(k / (Nl + 1));
  out[k] = psi_in[(int64_t)I * step + (int64_t)J * step * (N0 + 1)];
}

}  // namespace

int assemble_level(mgfem_ctx* c, int l, const double* psi_in, const double* chi_in) {
  Level& L = c->lv[l];
  const int N = L.N;
  const int64_t n = L.n, nc = (int64_t)N * N;
  const double h = (c->p.x_hi - c->p.x_lo) / N;
  const int tb = 256;
  double *raw = nullptr, *psi = nullptr, *lam = nullptr, *chi = nullptr;
  uint8_t* ct = nullptr;
  Stats* st = nullptr;  // statistics of the coarse grids are not reported
  MGFEM_HIP_TRY(ctx_alloc_t(c, &raw, n));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &psi, n));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &lam, nc));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &ct, nc));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &st, 1));
  if (chi_in) MGFEM_HIP_TRY(ctx_alloc_t(c, &chi, n));
  {
    Stats init{};
    init.min_theta_bits = 0x7ff0000000000000ull;
    MGFEM_HIP_TRY(hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, c->s));
  }
  MGFEM_HIP_TRY(ctx_alloc_t(c, &L.A, 9 * n));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &L.flags, n));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &L.cellcut, nc));
  hipLaunchKernelGGL(k_inject, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, c->s, psi_in, c->N, c->N / N, raw,
                     N);
  if (chi_in)
    hipLaunchKernelGGL(k_inject, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, c->s, chi_in, c->N, c->N / N,
                       chi, N);
  hipLaunchKernelGGL(k_snap, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, c->s, (const double*)raw, psi, n,
                     pow(h, c->p.snap_alpha), st);
  hipLaunchKernelGGL(k_classify, dim3((unsigned)((nc + tb - 1) / tb)), dim3(tb), 0, c->s, (const double*)psi,
                     (const double*)chi, N, c->p, h, ct, lam, L.cellcut, st);
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, c->s, (const double*)psi,
                     (const double*)chi, N, c->p, h, (const uint8_t*)ct, (const double*)lam, L.A, (double*)nullptr,
                     (double*)nullptr, (double*)nullptr, L.flags, st, 0, 0.0, (double*)nullptr);
  MGFEM_HIP_TRY(hipGetLastError());
  return MGFEM_OK;
}

int setup_geometry(mgfem_ctx* c, const double* psi_in, const double* chi_in) {
  const int N = c->N;
  // the global rule: one lambda for every cut cell, computed beforehand
  mgfem_params pk = c->p;
  if (pk.stab_rule == MGFEM_STAB_GLOBAL) {
    pk.stab_rule = MGFEM_STAB_FIXED;
    pk.lambda_fixed = c->lambda_global;
  }
  const bool stiff = c->op_kind == kOpStiffness;
  const int64_t n = (int64_t)(N + 1) * (N + 1), nc = (int64_t)N * N;
  Level& L0 = c->lv[0];
  MGFEM_HIP_TRY(ctx_alloc_t(c, &c->psi, n));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &c->cell_type, nc));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &c->cell_lambda, nc));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &c->M, 9 * n));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &c->G, 9 * n));
  if (chi_in) MGFEM_HIP_TRY(ctx_alloc_t(c, &c->GN, 9 * n));
  if (stiff) MGFEM_HIP_TRY(ctx_alloc_t(c, &c->Kp, 9 * n));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &L0.A, 9 * n));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &L0.flags, n));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &L0.cellcut, nc));
  const int tb = 256;
  double thr = pow(c->h, c->p.snap_alpha);
  hipLaunchKernelGGL(k_snap, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, c->s, psi_in, c->psi,
                     n, thr, c->stats);
  hipLaunchKernelGGL(k_classify, dim3((unsigned)((nc + tb - 1) / tb)), dim3(tb), 0, c->s, c->psi, chi_in, N,
                     pk, c->h, c->cell_type, c->cell_lambda, L0.cellcut, c->stats);
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, c->s, c->psi, chi_in, N,
                     pk, c->h, c->cell_type, c->cell_lambda, L0.A, c->M, c->G, c->GN, L0.flags,
                     c->stats, stiff ? 1 : 0, stiff ? kStiffnessShift : 0.0, c->Kp);
  MGFEM_HIP_TRY(hipGetLastError());
  return MGFEM_OK;
}

}  // namespace mgfem
