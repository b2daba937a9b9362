// Level-0 vector kernels around the cycle: the load vector F = M f + G g,
// residual norms of the convergence history (l-infinity, section 3.1, and l2),
// stencil products for the gradients, masks, copies and casts.  Rows marked
// as not stored are the interior Q1 stencil (8/3 centre, -1/3 neighbours).
#include <algorithm>
#include <cmath>

#include "mgfem_internal.h"

namespace mgfem {
namespace {


// the box kernels below run 256 x 4 nodes per block (a thread takes one
// column of four rows), so that every thread has four independent load chains
// in flight; block (x, y) writes the partial pair x + y * gridDim.x
constexpr int kNodesPerThread = 4;

// max that propagates NaN (so a diverged solve is reported, not hidden)
__device__ inline double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

template <class T>
struct LevelView {
  const T* A;
  const uint8_t* fl;
  T* x;
  T* b;
  T* r;
  int N, s;
  int64_t n;
};

template <class T>
__device__ inline T row_times_x(const LevelView<T>& v, int i, int j, int64_t k, uint8_t f, T& diag) {
  const T* x = v.x;
  if (f & kFlagStored) {
    const T* A = v.A;
    const int64_t n = v.n;
    diag = A[4 * n + k];
    T acc = diag * x[k];
    const bool w = i > 0, e = i < v.N, so = j > 0, no = j < v.N;
    if (so) {
      if (w) acc += A[k] * x[k - v.s - 1];
      acc += A[n + k] * x[k - v.s];
      if (e) acc += A[2 * n + k] * x[k - v.s + 1];
    }
    if (w) acc += A[3 * n + k] * x[k - 1];
    if (e) acc += A[5 * n + k] * x[k + 1];
    if (no) {
      if (w) acc += A[6 * n + k] * x[k + v.s - 1];
      acc += A[7 * n + k] * x[k + v.s];
      if (e) acc += A[8 * n + k] * x[k + v.s + 1];
    }
    return acc;
  }
  diag = T(8) / T(3);
  const T nb = (x[k - v.s - 1] + x[k - v.s] + x[k - v.s + 1]) + (x[k - 1] + x[k + 1]) +
               (x[k + v.s - 1] + x[k + v.s] + x[k + v.s + 1]);
  return diag * x[k] - nb * T(1.0 / 3.0);
}

// per-block (max |v|, sum v^2) of a block of 256 threads into part[2 b],
// part[2 b + 1]: a wave reduction, then the four waves in a fixed order
__device__ inline void block_pair(double mx, double sm, double* __restrict__ part) {
  __shared__ double smax[4], ssum[4];
  for (int o = 32; o > 0; o >>= 1) {
    mx = nanmax(mx, __shfl_xor(mx, o));
    sm += __shfl_xor(sm, o);
  }
  if ((threadIdx.x & 63) == 0) {
    smax[threadIdx.x >> 6] = mx;
    ssum[threadIdx.x >> 6] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      mx = nanmax(mx, smax[w]);
      sm += ssum[w];
    }
    const int b = blockIdx.x + blockIdx.y * gridDim.x;
    part[2 * b] = mx;
    part[2 * b + 1] = sm;
  }
}

// A block of the box kernels owns 256 x 4 nodes; the values its stencils read
// are staged in LDS with a halo of one (zero off the grid), every global load
// of the staging issued before the first is used: none sits under a branch
// (a node off the grid loads a clamped on-grid node and stores zero; the
// LDS area is padded to whole rounds of the block, kSNP), since a load under
// a branch waits for the ones before it.
constexpr int kBX = 256, kBY = kNodesPerThread, kSW = kBX + 2, kSH = kBY + 2, kSN = kSW * kSH;
constexpr int kSNP = (kSN + 255) / 256 * 256;

template <class Load>
__device__ inline void stage_box(double* __restrict__ sv, int bi, int bj, int N, int s, Load load) {
  constexpr int NU = kSNP / 256;
  double r[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int q = min(threadIdx.x + u * 256, kSN - 1);
    const int gi = min(max(bi - 1 + q % kSW, 0), N), gj = min(max(bj - 1 + q / kSW, 0), N);
    r[u] = load(gi + (int64_t)gj * s);
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int q = threadIdx.x + u * 256;
    const int gi = bi - 1 + q % kSW, gj = bj - 1 + q / kSW;
    const bool in = q < kSN && gi >= 0 && gj >= 0 && gi <= N && gj <= N;
    sv[q] = in ? r[u] : 0.0;
  }
  __syncthreads();
}

__device__ inline double box_neighbours(const double* sv, int q) {
  return (sv[q - kSW - 1] + sv[q - kSW] + sv[q - kSW + 1]) + (sv[q - 1] + sv[q + 1]) +
         (sv[q + kSW - 1] + sv[q + kSW] + sv[q + kSW + 1]);
}

// stored row times the staged values (the row's off-grid coefficients are zero)
__device__ inline double box_row(const double* __restrict__ A, int64_t n, int64_t k, const double* sv, int q) {
  double acc = A[4 * n + k] * sv[q];
  acc += A[k] * sv[q - kSW - 1];
  acc += A[n + k] * sv[q - kSW];
  acc += A[2 * n + k] * sv[q - kSW + 1];
  acc += A[3 * n + k] * sv[q - 1];
  acc += A[5 * n + k] * sv[q + 1];
  acc += A[6 * n + k] * sv[q + kSW - 1];
  acc += A[7 * n + k] * sv[q + kSW];
  acc += A[8 * n + k] * sv[q + kSW + 1];
  return acc;
}

// residual norms of level 0: per-block max |r| and sum r^2 (one node per
// thread, partials in block order: deterministic); optionally stores r
__global__ __launch_bounds__(256) void k_resnorm_partial(LevelView<double> v, const double* __restrict__ F,
                                                         double* r_out, int i0, int j0, int ni, int nj,
                                                         double* __restrict__ part) {
  __shared__ double sv[kSNP];
  const int bi = i0 + blockIdx.x * kBX, bj = j0 + blockIdx.y * kBY;
  const double* x = v.x;
  stage_box(sv, bi, bj, v.N, v.s, [&](int64_t k) { return x[k]; });
  double mx = 0.0, sm = 0.0;
  const int i = bi + threadIdx.x;
#pragma unroll
  for (int rep = 0; rep < kBY; ++rep) {
    const int j = bj + rep;
    if (i >= i0 + ni || j >= j0 + nj) continue;
    const int64_t k = i + (int64_t)j * v.s;
    const uint8_t f = v.fl[k];
    if (!(f & kFlagActive)) continue;
    const int q = threadIdx.x + 1 + (rep + 1) * kSW;
    const double ax = (f & kFlagStored) ? box_row(v.A, v.n, k, sv, q)
                                        : 8.0 / 3.0 * sv[q] - box_neighbours(sv, q) * (1.0 / 3.0);
    const double r = F[k] - ax;
    if (r_out) r_out[k] = r;
    mx = nanmax(mx, fabs(r));
    sm += r * r;
  }
  block_pair(mx, sm, part);
}

__global__ void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                              double* __restrict__ part) {
  double sm = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    sm += a[t] * b[t];
  block_pair(0.0, sm, part);
}

__global__ __launch_bounds__(1024) void k_reduce_final(const double* __restrict__ part, int nb,
                                                      double* __restrict__ out, double* host_out, double* seq) {
  __shared__ double smax[16], ssum[16];
  // pairs in chunks of 8 per thread, the loads of a chunk issued together (a
  // lane beyond nb reads pair 0 and drops it: loads under a branch would
  // wait for one another)
  constexpr int U = 8;
  double mx = 0.0, sm = 0.0;
  for (int base = 0; base < nb; base += U * 1024) {
    double lm[U], ls[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = base + threadIdx.x + u * 1024;
      const int tt = t < nb ? t : 0;
      lm[u] = part[2 * tt];
      ls[u] = part[2 * tt + 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = base + (int)threadIdx.x + u * 1024 < nb;
      mx = nanmax(mx, in ? lm[u] : 0.0);
      sm += in ? ls[u] : 0.0;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mx = nanmax(mx, __shfl_xor(mx, o));
    sm += __shfl_xor(sm, o);
  }
  if ((threadIdx.x & 63) == 0) {
    smax[threadIdx.x >> 6] = mx;
    ssum[threadIdx.x >> 6] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      mx = nanmax(mx, smax[w]);
      sm += ssum[w];
    }
    out[0] = mx;
    out[1] = sm;
    // straight to pinned host memory; the sequence number (counted on the
    // device, so a replayed graph still numbers its reductions) goes last
    const double q = seq[0] + 1.0;
    seq[0] = q;
    double* rec = host_out + 4 * (int)((long long)q % kRedSlots);
    rec[0] = mx;
    rec[1] = sm;
    __threadfence_system();
    rec[2] = q;
    __threadfence_system();
  }
}

// F = M f + G g (+ GN g_N on mixed boundaries; section 2, the discrete load)
// in two parts.  The vertices of cut cells (the rows that differ from the
// interior ones) take their M and G rows from one contiguous gathered array
// (18 values per vertex, in cut-list order; the GN rows, 9 per vertex, from a
// second one): k_cut_rows.  Every other node of the box of active nodes is done by
// k_rhs: an active row whose four cells are interior has the constant Q1 mass
// stencil h^2/36 [1 4 1; 4 16 4; 1 4 1] and no boundary term; k_rhs also
// reduces (max |F|, sum F^2) over all active nodes, reading F at the cut
// vertices, so k_cut_rows runs first.
__global__ void k_cut_rows(const int* __restrict__ cut_list, int ncut, const double* __restrict__ rows,
                           const double* __restrict__ x, const double* __restrict__ g,
                           const double* __restrict__ rows_n, const double* __restrict__ gn,
                           double* __restrict__ y, int N) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncut) return;
  const int s = N + 1;
  const int64_t k = cut_list[t];
  const int i = (int)(k % s), j = (int)(k / s);
  const double* r = rows + 18 * (int64_t)t;
  double acc = 0.0;
  for (int p = 0; p < 9; ++p) {
    const int ii = i + p % 3 - 1, jj = j + p / 3 - 1;
    if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
    const int64_t kk = ii + (int64_t)jj * s;
    const double m = r[p], gg = r[9 + p];
    if (m != 0.0) acc += m * x[kk];
    if (g && gg != 0.0) acc += gg * g[kk];
    if (gn) {
      const double w = rows_n[9 * (int64_t)t + p];
      if (w != 0.0) acc += w * gn[kk];
    }
  }
  y[k] = acc;
}

// y = GN x at the vertices of cut cells (GN is symmetric and vanishes
// elsewhere; y must be zero off them)
__global__ void k_cut_rows9(const int* __restrict__ cut_list, int ncut, const double* __restrict__ rows_n,
                            const double* __restrict__ x, double* __restrict__ y, int N) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncut) return;
  const int s = N + 1;
  const int64_t k = cut_list[t];
  const int i = (int)(k % s), j = (int)(k / s);
  double acc = 0.0;
  for (int p = 0; p < 9; ++p) {
    const int ii = i + p % 3 - 1, jj = j + p / 3 - 1;
    if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
    const double w = rows_n[9 * (int64_t)t + p];
    if (w != 0.0) acc += w * x[ii + (int64_t)jj * s];
  }
  y[k] = acc;
}

// y = G^T x at the vertices of cut cells (G couples only vertices of one cut
// cell, so G^T x vanishes elsewhere): the coefficient of column k in row kk
// is plane 8 - p of row kk, found through the row's cut-list position
__global__ void k_cut_rows_gt(const int* __restrict__ cut_list, int ncut, const int* __restrict__ cutpos,
                              const double* __restrict__ rows, const double* __restrict__ x,
                              double* __restrict__ y, int N) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncut) return;
  const int s = N + 1;
  const int64_t k = cut_list[t];
  const int i = (int)(k % s), j = (int)(k / s);
  double acc = 0.0;
  for (int p = 0; p < 9; ++p) {
    const int ii = i + p % 3 - 1, jj = j + p / 3 - 1;
    if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
    const int64_t kk = ii + (int64_t)jj * s;
    const int q = cutpos[kk];
    if (q < 0) continue;
    const double a = rows[18 * (int64_t)q + 9 + (8 - p)];
    if (a != 0.0) acc += a * x[kk];
  }
  y[k] = acc;
}

__device__ inline double mass_row(const double* sv, int q, double hh36) {
  const double corners = (sv[q - kSW - 1] + sv[q - kSW + 1]) + (sv[q + kSW - 1] + sv[q + kSW + 1]);
  const double edges = (sv[q - kSW] + sv[q + kSW]) + (sv[q - 1] + sv[q + 1]);
  return hh36 * (16.0 * sv[q] + 4.0 * edges + corners);
}

// a stored row that is not a cut-cell vertex (none arise from the assembly;
// kept so that every row is covered): from the full planes
__device__ inline double plane_row(const double* __restrict__ S, const double* __restrict__ x, int64_t n,
                                   int64_t k, int i, int j, int N, int s) {
  double acc = 0.0;
  for (int p = 0; p < 9; ++p) {
    const int ii = i + p % 3 - 1, jj = j + p / 3 - 1;
    if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
    const double a = S[p * n + k];
    if (a != 0.0) acc += a * x[ii + (int64_t)jj * s];
  }
  return acc;
}

__global__ __launch_bounds__(256) void k_rhs(const double* __restrict__ M, const double* __restrict__ G,
                                             const double* __restrict__ GN, const uint8_t* __restrict__ fl,
                                             const double* __restrict__ f, const double* __restrict__ g,
                                             const double* __restrict__ gn, double* __restrict__ F, int N,
                                             double hh36, int i0, int j0, int ni, int nj,
                                             double* __restrict__ part) {
  __shared__ double sv[kSNP];
  const int s = N + 1;
  const int64_t n = (int64_t)s * s;
  const int bi = i0 + blockIdx.x * kBX, bj = j0 + blockIdx.y * kBY;
  stage_box(sv, bi, bj, N, s, [&](int64_t k) { return f[k]; });
  double mx = 0.0, sm = 0.0;
  const int i = bi + threadIdx.x;
#pragma unroll
  for (int rep = 0; rep < kBY; ++rep) {
    const int j = bj + rep;
    if (i >= i0 + ni || j >= j0 + nj) continue;
    const int64_t k = i + (int64_t)j * s;
    const uint8_t fk = fl[k];
    double acc = 0.0;
    if (fk & kFlagActive) {
      if (!(fk & kFlagStored)) acc = mass_row(sv, threadIdx.x + 1 + (rep + 1) * kSW, hh36);
      else if (fk & kFlagCut) acc = F[k];  // from k_cut_rows
      else {
        acc = plane_row(M, f, n, k, i, j, N, s) + plane_row(G, g, n, k, i, j, N, s);
        if (gn) acc += plane_row(GN, gn, n, k, i, j, N, s);
      }
    }
    if (!(fk & kFlagActive) || !(fk & kFlagStored) || !(fk & kFlagCut)) F[k] = acc;
    mx = nanmax(mx, fabs(acc));
    sm += acc * acc;
  }
  block_pair(mx, sm, part);
}

// y = M x on the whole grid (zero off the box of active nodes and at inactive
// nodes); the rows of cut-cell vertices are left to k_cut_rows
__global__ __launch_bounds__(256) void k_mass_grid(const double* __restrict__ M, const uint8_t* __restrict__ fl,
                                                   const double* __restrict__ x, double* __restrict__ y, int N,
                                                   double hh36, int i0, int j0, int i1, int j1) {
  __shared__ double sv[kSNP];
  const int s = N + 1;
  const int64_t n = (int64_t)s * s;
  const int bi = blockIdx.x * kBX, bj = blockIdx.y * kBY;
  const bool touches = bi <= i1 && bi + kBX - 1 >= i0 && bj <= j1 && bj + kBY - 1 >= j0;  // uniform
  if (touches) stage_box(sv, bi, bj, N, s, [&](int64_t k) { return x[k]; });
  const int i = bi + threadIdx.x;
#pragma unroll
  for (int rep = 0; rep < kBY; ++rep) {
    const int j = bj + rep;
    if (i > N || j > N) continue;
    const int64_t k = i + (int64_t)j * s;
    if (!touches || i < i0 || i > i1 || j < j0 || j > j1) {
      y[k] = 0.0;
      continue;
    }
    const uint8_t fk = fl[k];
    if (!(fk & kFlagActive)) y[k] = 0.0;
    else if (!(fk & kFlagStored)) y[k] = mass_row(sv, threadIdx.x + 1 + (rep + 1) * kSW, hh36);
    else if (!(fk & kFlagCut)) y[k] = plane_row(M, x, n, k, i, j, N, s);
  }
}

// Outer step of the mixed-precision solve, on the box of active nodes:
// u_new = u + e (e: the float correction, null for none), r = F - A u_new in
// float64, the float copy of r as the next inner right-hand side, a zero
// float start iterate for the next inner cycle, and (max |r|, sum r^2).
// u_new goes to a second buffer, so every thread reads the old u.
__global__ __launch_bounds__(256) void k_outer(LevelView<double> v, const double* __restrict__ F,
                                               const double* __restrict__ u, const float* __restrict__ e,
                                               double* __restrict__ u_out, float* __restrict__ r32,
                                               float* __restrict__ z32, int i0, int j0, int ni, int nj,
                                               double* __restrict__ part) {
  __shared__ double sv[kSNP];
  const int bi = i0 + blockIdx.x * kBX, bj = j0 + blockIdx.y * kBY;
  if (e) stage_box(sv, bi, bj, v.N, v.s, [&](int64_t k) { return u[k] + (double)e[k]; });
  else stage_box(sv, bi, bj, v.N, v.s, [&](int64_t k) { return u[k]; });
  double mx = 0.0, sm = 0.0;
  const int i = bi + threadIdx.x;
#pragma unroll
  for (int rep = 0; rep < kBY; ++rep) {
    const int j = bj + rep;
    if (i >= i0 + ni || j >= j0 + nj) continue;
    const int64_t k = i + (int64_t)j * v.s;
    const uint8_t f = v.fl[k];
    if (!(f & kFlagActive)) continue;
    const int q = threadIdx.x + 1 + (rep + 1) * kSW;
    const double uk = sv[q];
    const double ax = (f & kFlagStored) ? box_row(v.A, v.n, k, sv, q)
                                        : 8.0 / 3.0 * uk - box_neighbours(sv, q) * (1.0 / 3.0);
    const double r = F[k] - ax;
    if (u_out) u_out[k] = uk;
    r32[k] = (float)r;
    z32[k] = 0.0f;
    mx = nanmax(mx, fabs(r));
    sm += r * r;
  }
  block_pair(mx, sm, part);
}

// The same outer step over the level's sweep tiles that hold an active node
// (TW x TH cores, in the tile list of the sweeps) instead of the whole box
// of active nodes: blocks of the box with no active node cost no loads.
// Each block stages its core plus a ring of one (u + e, zero off the grid)
// with every load issued before the first is used; the arithmetic of a node
// is that of k_outer, operation for operation.  Partials in tile-list order.
template <int TW, int TH, bool E>
__global__ __launch_bounds__(256) void k_outer_tiles(LevelView<double> v, const int* __restrict__ tiles, int ntx,
                                                     int i0, int j0, int i1, int j1, const double* __restrict__ F,
                                                     const double* __restrict__ u, const float* __restrict__ e,
                                                     double* __restrict__ u_out, float* __restrict__ r32,
                                                     float* __restrict__ z32, double* __restrict__ part) {
  constexpr int SW = TW + 2, SN = SW * (TH + 2), NU = (SN + 255) / 256, NC = TW * TH / 256;
  __shared__ double sv[NU * 256];  // the region, padded to whole rounds of the block
  const int tile = tiles[blockIdx.x];
  const int bi = i0 + (tile % ntx) * TW, bj = j0 + (tile / ntx) * TH;
  // Every load of the block issued before any is used, none under a branch
  // (a node off the grid or beyond the box reads a clamped on-grid node and
  // drops it): the staged u + e, then the flags and F of this thread's core
  // nodes.
  double ru[NU];
  float re[NU];
#pragma unroll
  for (int w = 0; w < NU; ++w) {
    const int q = min(threadIdx.x + w * 256, SN - 1);
    const int gi = min(max(bi - 1 + q % SW, 0), v.N), gj = min(max(bj - 1 + q / SW, 0), v.N);
    const int64_t k = gi + (int64_t)gj * v.s;
    ru[w] = u[k];
    re[w] = E ? e[k] : 0.0f;
  }
  uint8_t fk[NC];
  double Fk[NC];
#pragma unroll
  for (int w = 0; w < NC; ++w) {
    const int c = threadIdx.x + w * 256;
    const int i = bi + c % TW, j = bj + c / TW;
    const int64_t k = min(i, v.N) + (int64_t)min(j, v.N) * v.s;
    fk[w] = v.fl[k] & ((i <= i1 && j <= j1) ? 0xff : 0);
    Fk[w] = F[k];
  }
#pragma unroll
  for (int w = 0; w < NU; ++w) {
    const int q = threadIdx.x + w * 256;
    const int gi = bi - 1 + q % SW, gj = bj - 1 + q / SW;
    const bool in = gi >= 0 && gj >= 0 && gi <= v.N && gj <= v.N;
    sv[q] = in ? (E ? ru[w] + (double)re[w] : ru[w]) : 0.0;
  }
  __syncthreads();
  double mx = 0.0, sm = 0.0;
#pragma unroll
  for (int w = 0; w < NC; ++w) {
    const int c = threadIdx.x + w * 256;
    const uint8_t f = fk[w];
    if (!(f & kFlagActive)) continue;
    const int64_t k = (bi + c % TW) + (int64_t)(bj + c / TW) * v.s;
    const int q = (c % TW + 1) + (c / TW + 1) * SW;
    const double uk = sv[q];
    double ax;
    if (f & kFlagStored) {
      const int64_t n = v.n;
      ax = v.A[4 * n + k] * sv[q];
      ax += v.A[k] * sv[q - SW - 1];
      ax += v.A[n + k] * sv[q - SW];
      ax += v.A[2 * n + k] * sv[q - SW + 1];
      ax += v.A[3 * n + k] * sv[q - 1];
      ax += v.A[5 * n + k] * sv[q + 1];
      ax += v.A[6 * n + k] * sv[q + SW - 1];
      ax += v.A[7 * n + k] * sv[q + SW];
      ax += v.A[8 * n + k] * sv[q + SW + 1];
    } else {
      const double nb = (sv[q - SW - 1] + sv[q - SW] + sv[q - SW + 1]) + (sv[q - 1] + sv[q + 1]) +
                        (sv[q + SW - 1] + sv[q + SW] + sv[q + SW + 1]);
      ax = 8.0 / 3.0 * uk - nb * (1.0 / 3.0);
    }
    const double r = Fk[w] - ax;
    if (u_out) u_out[k] = uk;
    r32[k] = (float)r;
    z32[k] = 0.0f;
    mx = nanmax(mx, fabs(r));
    sm += r * r;
  }
  block_pair(mx, sm, part);
}

__global__ void k_mask(const uint8_t* __restrict__ fl, double* __restrict__ u, int64_t n, int zero_all) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (zero_all || !(fl[k] & kFlagActive)) u[k] = 0.0;
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) d[k] = s[k];
}

inline unsigned nblk(int64_t n, int tb) { return (unsigned)((n + tb - 1) / tb); }

}  // namespace

void launch_rhs(mgfem_ctx* c, const double* f, const double* g, const double* gN, double* F) {
  const Level& L = c->lv[0];
  const int ncut = L.cut_off[4];
  if (!c->GN) gN = nullptr;  // no Neumann segment: the Neumann data are not read
  if (ncut > 0)
    hipLaunchKernelGGL(k_cut_rows, dim3(nblk(ncut, 256)), dim3(256), 0, c->s, L.cut_list, ncut, c->cut_rows, f, g,
                       (const double*)c->cut_rows_n, gN, F, c->N);
  const int ni = L.bbox[1] - L.bbox[0] + 1, nj = L.bbox[3] - L.bbox[2] + 1;
  const dim3 grid((unsigned)std::max(1, (ni + 255) / 256), (unsigned)std::max(1, (nj + 3) / 4));
  const int nb = (int)(grid.x * grid.y);
  hipLaunchKernelGGL(k_rhs, grid, dim3(256), 0, c->s, c->M, c->G, (const double*)c->GN, L.flags, f, g, gN, F, c->N,
                     c->h * c->h / 36.0, L.bbox[0], L.bbox[2], ni, nj, c->red_partial);
  c->red_seq += 1.0;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, c->s, c->red_partial, nb, c->red_out, c->red_host,
                     c->red_seq_dev);
}

void launch_outer(mgfem_ctx* c, const double* u, const float* e, double* u_out, float* r32, float* z32) {
  Level& L = c->lv[0];
  LevelView<double> v{L.A, L.flags, nullptr, nullptr, nullptr, L.N, L.stride, L.n};
  if (L.tiles && L.ntiles > 0) {
    // over the active sweep tiles of level 0, in their shape
    const int shape = sweep_shape(c, 0);
    const int TW = shape == kShapeSmall ? 16 : 64, TH = shape == kShapeFinest ? 32 : 16;
    const int ntx = (L.bbox[1] - L.bbox[0] + TW) / TW;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(L.ntiles), dim3(256), 0, c->s, v, (const int*)L.tiles, ntx, L.bbox[0],
                         L.bbox[2], L.bbox[1], L.bbox[3], (const double*)L.b, u, e, u_out, r32, z32, c->sweep_part);
    };
    if (shape == kShapeFinest) e ? go(k_outer_tiles<64, 32, true>) : go(k_outer_tiles<64, 32, false>);
    else if (shape == kShapeLarge) e ? go(k_outer_tiles<64, 16, true>) : go(k_outer_tiles<64, 16, false>);
    else e ? go(k_outer_tiles<16, 16, true>) : go(k_outer_tiles<16, 16, false>);
    c->red_seq += 1.0;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, c->s, (const double*)c->sweep_part, L.ntiles,
                       c->red_out, c->red_host, c->red_seq_dev);
    return;
  }
  const int ni = L.bbox[1] - L.bbox[0] + 1, nj = L.bbox[3] - L.bbox[2] + 1;
  const dim3 grid((unsigned)std::max(1, (ni + 255) / 256), (unsigned)std::max(1, (nj + 3) / 4));
  const int nb = (int)(grid.x * grid.y);
  hipLaunchKernelGGL(k_outer, grid, dim3(256), 0, c->s, v, (const double*)L.b, u, e, u_out, r32, z32,
                     L.bbox[0], L.bbox[2], ni, nj, c->red_partial);
  c->red_seq += 1.0;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, c->s, c->red_partial, nb, c->red_out, c->red_host,
                     c->red_seq_dev);
}

namespace {
// the M and G rows (and GN rows) of every cut-cell vertex of level 0, in cut-list order
__global__ void k_gather_cut_rows(const int* __restrict__ cut_list, int ncut, const double* __restrict__ M,
                                  const double* __restrict__ G, const double* __restrict__ GN,
                                  const double* __restrict__ Kp, int64_t n, double* __restrict__ rows,
                                  double* __restrict__ rows_n, double* __restrict__ rows_k) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncut) return;
  const int64_t k = cut_list[t];
  for (int p = 0; p < 9; ++p) {
    rows[18 * (int64_t)t + p] = M[p * n + k];
    rows[18 * (int64_t)t + 9 + p] = G[p * n + k];
    if (GN) rows_n[9 * (int64_t)t + p] = GN[p * n + k];
    if (Kp) rows_k[9 * (int64_t)t + p] = Kp[p * n + k];
  }
}
}  // namespace

int build_cut_rows(mgfem_ctx* c) {
  const Level& L = c->lv[0];
  const int ncut = L.cut_off[4];
  MGFEM_HIP_TRY(ctx_alloc_t(c, &c->cut_rows, 18 * (size_t)std::max(1, ncut)));
  if (c->GN) MGFEM_HIP_TRY(ctx_alloc_t(c, &c->cut_rows_n, 9 * (size_t)std::max(1, ncut)));
  if (c->Kp) MGFEM_HIP_TRY(ctx_alloc_t(c, &c->cut_rows_k, 9 * (size_t)std::max(1, ncut)));
  if (ncut > 0)
    hipLaunchKernelGGL(k_gather_cut_rows, dim3(nblk(ncut, 256)), dim3(256), 0, c->s, L.cut_list, ncut, c->M, c->G,
                       (const double*)c->GN, (const double*)c->Kp, L.n, c->cut_rows, c->cut_rows_n,
                       c->cut_rows_k);
  MGFEM_HIP_TRY(hipGetLastError());
  return MGFEM_OK;
}

void launch_mass_apply(mgfem_ctx* c, const double* x, double* y) {
  const Level& L = c->lv[0];
  const int N = c->N;
  const dim3 grid((unsigned)((N + 1 + kBX - 1) / kBX), (unsigned)((N + 1 + kBY - 1) / kBY));
  hipLaunchKernelGGL(k_mass_grid, grid, dim3(256), 0, c->s, c->M, L.flags, x, y, N, c->h * c->h / 36.0,
                     L.bbox[0], L.bbox[2], L.bbox[1], L.bbox[3]);
  const int ncut = L.cut_off[4];
  if (ncut > 0)
    hipLaunchKernelGGL(k_cut_rows, dim3(nblk(ncut, 256)), dim3(256), 0, c->s, L.cut_list, ncut, c->cut_rows, x,
                       (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, y, N);
}

void launch_k_apply(mgfem_ctx* c, const double* x, double* y) {
  const Level& L = c->lv[0];
  launch_zero(c, y, L.n);
  const int ncut = L.cut_off[4];
  if (c->Kp && ncut > 0)
    hipLaunchKernelGGL(k_cut_rows9, dim3(nblk(ncut, 256)), dim3(256), 0, c->s, L.cut_list, ncut,
                       (const double*)c->cut_rows_k, x, y, c->N);
}

void launch_gn_apply(mgfem_ctx* c, const double* x, double* y) {
  const Level& L = c->lv[0];
  launch_zero(c, y, L.n);
  const int ncut = L.cut_off[4];
  if (c->GN && ncut > 0)
    hipLaunchKernelGGL(k_cut_rows9, dim3(nblk(ncut, 256)), dim3(256), 0, c->s, L.cut_list, ncut,
                       (const double*)c->cut_rows_n, x, y, c->N);
}

void launch_gt_apply(mgfem_ctx* c, const double* x, double* y) {
  const Level& L = c->lv[0];
  launch_zero(c, y, L.n);
  const int ncut = L.cut_off[4];
  if (ncut > 0)
    hipLaunchKernelGGL(k_cut_rows_gt, dim3(nblk(ncut, 256)), dim3(256), 0, c->s, L.cut_list, ncut, L.cutpos,
                       c->cut_rows, x, y, c->N);
}

void launch_mask_inactive(mgfem_ctx* c, double* u) {
  const int64_t n = c->lv[0].n;
  hipLaunchKernelGGL(k_mask, dim3(nblk(n, 256)), dim3(256), 0, c->s, c->lv[0].flags, u, n, 0);
}

void launch_zero(mgfem_ctx* c, double* p, int64_t n) {
  hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, c->s, p, n, 0.0);
}

void launch_copy(mgfem_ctx* c, double* dst, const double* src, int64_t n) {
  hipLaunchKernelGGL(k_copy, dim3(nblk(n, 256)), dim3(256), 0, c->s, dst, src, n);
}

// ||F - A u||_inf and ||.||_2^2 of level 0 into c->red_out[0..1]; r_out optional
void launch_residual_norm(mgfem_ctx* c, const double* F, const double* u, double* r_out) {
  Level& L = c->lv[0];
  LevelView<double> v{L.A, L.flags, const_cast<double*>(u), nullptr, nullptr, L.N, L.stride, L.n};
  const int ni = L.bbox[1] - L.bbox[0] + 1, nj = L.bbox[3] - L.bbox[2] + 1;
  const dim3 grid((unsigned)std::max(1, (ni + 255) / 256), (unsigned)std::max(1, (nj + 3) / 4));
  const int nb = (int)(grid.x * grid.y);
  hipLaunchKernelGGL(k_resnorm_partial, grid, dim3(256), 0, c->s, v, F, r_out, L.bbox[0],
                     L.bbox[2], ni, nj, c->red_partial);
  c->red_seq += 1.0;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, c->s, c->red_partial, nb, c->red_out, c->red_host,
                     c->red_seq_dev);
}

void launch_dot_reduce(mgfem_ctx* c, const double* a, const double* b) {
  const int64_t n = c->lv[0].n;
  const int nb = (int)std::min<int64_t>(kDotBlocks, (n + 255) / 256);  // grid-stride beyond
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(256), 0, c->s, a, b, n, c->red_partial);
  c->red_seq += 1.0;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, c->s, c->red_partial, nb, c->red_out, c->red_host,
                     c->red_seq_dev);
}

}  // namespace mgfem

namespace mgfem {
namespace {
__global__ void k_sub(double* __restrict__ d, const double* __restrict__ a, const double* __restrict__ b,
                      const uint8_t* __restrict__ fl, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) d[k] = (fl[k] & kFlagActive) ? a[k] - b[k] : 0.0;
}
__global__ void k_u8_to_f64(const uint8_t* __restrict__ s, double* __restrict__ d, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) d[k] = (double)s[k];
}
inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }
}  // namespace

namespace {
// dst = src (src null: 0) on the box [i0, i0+ni) x [j0, j0+nj) of a grid with row stride s
__global__ void k_box_copy(double* __restrict__ dst, const double* __restrict__ src, int s, int i0, int j0,
                           int ni, int nj) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= ni || j >= nj) return;
  const int64_t k = (i0 + i) + (int64_t)(j0 + j) * s;
  dst[k] = src ? src[k] : 0.0;
}
// every node of dst: src inside the box, 0 outside
__global__ void k_export(double* __restrict__ dst, const double* __restrict__ src, int s, int i0, int j0, int i1,
                         int j1, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = (int)(k % s), j = (int)(k / s);
  dst[k] = (i >= i0 && i <= i1 && j >= j0 && j <= j1) ? src[k] : 0.0;
}
}  // namespace

// ---------------------------------------------------------------------------
// Level-0 kernels of batched solves: one TeamL0 entry per problem, work items
// (problem, block).  The arithmetic is that of k_cut_rows, k_rhs, k_outer and
// k_export above.
// ---------------------------------------------------------------------------
namespace {

// per-block (max, sum) into out[0], out[1]
__device__ inline void block_pair_to(double mx, double sm, double* __restrict__ out) {
  __shared__ double smax[4], ssum[4];
  for (int o = 32; o > 0; o >>= 1) {
    mx = nanmax(mx, __shfl_xor(mx, o));
    sm += __shfl_xor(sm, o);
  }
  if ((threadIdx.x & 63) == 0) {
    smax[threadIdx.x >> 6] = mx;
    ssum[threadIdx.x >> 6] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      mx = nanmax(mx, smax[w]);
      sm += ssum[w];
    }
    out[0] = mx;
    out[1] = sm;
  }
}

__global__ __launch_bounds__(256) void k_team_cut_rows(const TeamL0* __restrict__ tab, const int2* __restrict__ work,
                                                       int nwork) {
  if ((int)blockIdx.x >= nwork) return;
  const int2 w = work[blockIdx.x];
  const TeamL0& e = tab[w.x];
  const int t = w.y * 256 + threadIdx.x;
  if (t >= e.ncut) return;
  const int N = e.N, s = e.s;
  const int64_t k = e.cut_list[t];
  const int i = (int)(k % s), j = (int)(k / s);
  const double* r = e.cut_rows + 18 * (int64_t)t;
  double acc = 0.0;
  for (int p = 0; p < 9; ++p) {
    const int ii = i + p % 3 - 1, jj = j + p / 3 - 1;
    if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
    const int64_t kk = ii + (int64_t)jj * s;
    const double m = r[p], gg = r[9 + p];
    if (m != 0.0) acc += m * e.f[kk];
    if (gg != 0.0) acc += gg * e.g[kk];
  }
  e.F[k] = acc;
}

__global__ __launch_bounds__(256) void k_team_rhs(const TeamL0* __restrict__ tab, const int2* __restrict__ work,
                                                  int nwork) {
  __shared__ double sv[kSNP];
  if ((int)blockIdx.x >= nwork) return;
  const int2 w = work[blockIdx.x];
  const TeamL0& e = tab[w.x];
  const int N = e.N, s = e.s;
  const int bi = e.i0 + (w.y % e.gx) * kBX, bj = e.j0 + (w.y / e.gx) * kBY;
  const double* f = e.f;
  stage_box(sv, bi, bj, N, s, [&](int64_t k) { return f[k]; });
  double mx = 0.0, sm = 0.0;
  const int i = bi + threadIdx.x;
#pragma unroll
  for (int rep = 0; rep < kBY; ++rep) {
    const int j = bj + rep;
    if (i >= e.i0 + e.ni || j >= e.j0 + e.nj) continue;
    const int64_t k = i + (int64_t)j * s;
    const uint8_t fk = e.fl[k];
    double acc = 0.0;
    if (fk & kFlagActive) {
      if (!(fk & kFlagStored)) acc = mass_row(sv, threadIdx.x + 1 + (rep + 1) * kSW, e.h36);
      else if (fk & kFlagCut) acc = e.F[k];  // from k_team_cut_rows
      else acc = plane_row(e.M, f, e.n, k, i, j, N, s) + plane_row(e.G, e.g, e.n, k, i, j, N, s);
    }
    if (!(fk & kFlagActive) || !(fk & kFlagStored) || !(fk & kFlagCut)) e.F[k] = acc;
    mx = nanmax(mx, fabs(acc));
    sm += acc * acc;
  }
  block_pair_to(mx, sm, e.part + 2 * w.y);
}

// first = 1: the step from u = 0 (r = F; u's buffer 0 set to 0 on the active
// nodes); else u_new = U[upar] + E[epar] into U[1 - upar]
__global__ __launch_bounds__(256) void k_team_outer(const TeamL0* __restrict__ tab, const int2* __restrict__ work,
                                                    int nwork, int upar, int epar, int first) {
  __shared__ double sv[kSNP];
  if ((int)blockIdx.x >= nwork) return;
  const int2 w = work[blockIdx.x];
  const TeamL0& e = tab[w.x];
  const int bi = e.i0 + (w.y % e.gx) * kBX, bj = e.j0 + (w.y / e.gx) * kBY;
  const double* u = e.U[upar];
  const float* ev = e.E[epar];
  if (first) stage_box(sv, bi, bj, e.N, e.s, [&](int64_t) { return 0.0; });
  else stage_box(sv, bi, bj, e.N, e.s, [&](int64_t k) { return u[k] + (double)ev[k]; });
  double* u_out = first ? e.U[0] : e.U[1 - upar];
  float* z32 = first ? e.E[0] : e.E[1 - epar];
  double mx = 0.0, sm = 0.0;
  const int i = bi + threadIdx.x;
#pragma unroll
  for (int rep = 0; rep < kBY; ++rep) {
    const int j = bj + rep;
    if (i >= e.i0 + e.ni || j >= e.j0 + e.nj) continue;
    const int64_t k = i + (int64_t)j * e.s;
    const uint8_t f = e.fl[k];
    if (!(f & kFlagActive)) continue;
    const int q = threadIdx.x + 1 + (rep + 1) * kSW;
    const double uk = sv[q];
    const double ax = (f & kFlagStored) ? box_row(e.A, e.n, k, sv, q)
                                        : 8.0 / 3.0 * uk - box_neighbours(sv, q) * (1.0 / 3.0);
    const double r = e.F[k] - ax;
    u_out[k] = uk;
    e.r32[k] = (float)r;
    z32[k] = 0.0f;
    mx = nanmax(mx, fabs(r));
    sm += r * r;
  }
  block_pair_to(mx, sm, e.part + 2 * w.y);
}

__global__ __launch_bounds__(256) void k_team_export(const TeamL0* __restrict__ tab, const int2* __restrict__ work,
                                                     int nwork) {
  if ((int)blockIdx.x >= nwork) return;
  const int2 w = work[blockIdx.x];
  const TeamL0& e = tab[w.x];
  const int64_t k = w.y * (int64_t)256 + threadIdx.x;
  if (k >= e.n) return;
  const int i = (int)(k % e.s), j = (int)(k / e.s);
  const bool in = i >= e.i0 && i < e.i0 + e.ni && j >= e.j0 && j < e.j0 + e.nj;
  e.u_out[k] = in ? e.U[e.ucur][k] : 0.0;
}

// one workgroup per listed problem: its box partials in block order
__global__ __launch_bounds__(256) void k_team_reduce(const TeamL0* __restrict__ tab, const int* __restrict__ probs,
                                                     double* __restrict__ out) {
  const int p = probs[blockIdx.x];
  const TeamL0& e = tab[p];
  double mx = 0.0, sm = 0.0;
  for (int q = threadIdx.x; q < e.nb; q += blockDim.x) {
    mx = nanmax(mx, e.part[2 * q]);
    sm += e.part[2 * q + 1];
  }
  block_pair_to(mx, sm, out + 2 * p);
}

}  // namespace

void team_l0_entry(mgfem_ctx* m, TeamL0* out) {
  const Level& L = m->lv[0];
  TeamL0 e{};
  e.A = L.A;
  e.fl = L.flags;
  e.N = L.N;
  e.s = L.stride;
  e.n = L.n;
  e.M = m->M;
  e.G = m->G;
  e.h36 = m->h * m->h / 36.0;
  e.cut_list = L.cut_list;
  e.ncut = L.cut_off[4];
  e.cut_rows = m->cut_rows;
  e.F = m->F;
  e.U[0] = m->x0;
  e.U[1] = L.X[1];
  e.E[0] = L.X32[0];
  e.E[1] = L.X32[1];
  e.r32 = L.b32;
  e.i0 = L.bbox[0];
  e.j0 = L.bbox[2];
  e.ni = std::max(0, L.bbox[1] - L.bbox[0] + 1);
  e.nj = std::max(0, L.bbox[3] - L.bbox[2] + 1);
  e.gx = std::max(1, (e.ni + kBX - 1) / kBX);
  e.nb = e.gx * std::max(1, (e.nj + kBY - 1) / kBY);
  e.part = m->red_partial;
  *out = e;
}

int team_l0_units(const TeamL0& e, int kind) {
  switch (kind) {
    case kTeamCutRows: return (e.ncut + 255) / 256;
    case kTeamRhs:
    case kTeamOuterFirst:
    case kTeamOuter: return e.ni > 0 && e.nj > 0 ? e.nb : 0;
    case kTeamExport: return (int)((e.n + 255) / 256);
  }
  return 0;
}

void team_l0_launch(hipStream_t s, int kind, const TeamL0* tab, const int2* work, int nwork, int upar, int epar) {
  if (nwork <= 0) return;
  switch (kind) {
    case kTeamCutRows: hipLaunchKernelGGL(k_team_cut_rows, dim3(nwork), dim3(256), 0, s, tab, work, nwork); break;
    case kTeamRhs: hipLaunchKernelGGL(k_team_rhs, dim3(nwork), dim3(256), 0, s, tab, work, nwork); break;
    case kTeamOuterFirst:
      hipLaunchKernelGGL(k_team_outer, dim3(nwork), dim3(256), 0, s, tab, work, nwork, 0, 0, 1);
      break;
    case kTeamOuter:
      hipLaunchKernelGGL(k_team_outer, dim3(nwork), dim3(256), 0, s, tab, work, nwork, upar, epar, 0);
      break;
    case kTeamExport: hipLaunchKernelGGL(k_team_export, dim3(nwork), dim3(256), 0, s, tab, work, nwork); break;
  }
}

void team_reduce(hipStream_t s, const TeamL0* tab, const int* probs, int nprobs, double* out) {
  if (nprobs > 0) hipLaunchKernelGGL(k_team_reduce, dim3(nprobs), dim3(256), 0, s, tab, probs, out);
}

void launch_box_copy(mgfem_ctx* c, double* dst, const double* src) {
  const Level& L = c->lv[0];
  const int ni = L.bbox[1] - L.bbox[0] + 1, nj = L.bbox[3] - L.bbox[2] + 1;
  if (ni <= 0 || nj <= 0) return;
  hipLaunchKernelGGL(k_box_copy, dim3((ni + 63) / 64, (nj + 3) / 4), dim3(64, 4), 0, c->s, dst, src, L.stride,
                     L.bbox[0], L.bbox[2], ni, nj);
}
void launch_export(mgfem_ctx* c, double* dst, const double* src) {
  const Level& L = c->lv[0];
  hipLaunchKernelGGL(k_export, dim3(nb256(L.n)), dim3(256), 0, c->s, dst, src, L.stride, L.bbox[0], L.bbox[2],
                     L.bbox[1], L.bbox[3], L.n);
}

void launch_sub_active(mgfem_ctx* c, double* d, const double* a, const double* b) {
  const int64_t n = c->lv[0].n;
  hipLaunchKernelGGL(k_sub, dim3(nb256(n)), dim3(256), 0, c->s, d, a, b, c->lv[0].flags, n);
}
void launch_u8_to_f64(mgfem_ctx* c, const uint8_t* s, double* d, int64_t n) {
  hipLaunchKernelGGL(k_u8_to_f64, dim3(nb256(n)), dim3(256), 0, c->s, s, d, n);
}
}  // namespace mgfem
