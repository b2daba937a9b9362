// Level-0 vector kernels around the cycle: the load vector F = M f + G g,
// residual norms of the convergence history (l-infinity, section 3.1, and l2),
// stencil products for the gradients, masks, copies and casts.  Rows marked
// as not stored are the interior Q1 stencil (8/3 centre, -1/3 neighbours).
#include <algorithm>
#include <cmath>

#include "mgfem_internal.h"

namespace mgfem {
namespace {


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
  return diag * x[k] - nb / T(3);
}

// residual norms of level 0: per-block max |r| and sum r^2 (fixed block count,
// fixed order: deterministic); optionally stores r
__global__ void k_resnorm_partial(LevelView<double> v, const double* __restrict__ F, double* r_out,
                                  int i0, int j0, int ni, int nj, double* __restrict__ part) {
  __shared__ double smax[256], ssum[256];
  double mx = 0.0, sm = 0.0;
  const int64_t tot = (int64_t)ni * nj;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = i0 + (int)(t % ni), j = j0 + (int)(t / ni);
    const int64_t k = i + (int64_t)j * v.s;
    const uint8_t f = v.fl[k];
    if (!(f & kFlagActive)) continue;
    double diag;
    const double r = F[k] - row_times_x(v, i, j, k, f, diag);
    if (r_out) r_out[k] = r;
    mx = nanmax(mx, fabs(r));
    sm += r * r;
  }
  smax[threadIdx.x] = mx;
  ssum[threadIdx.x] = sm;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      smax[threadIdx.x] = nanmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      ssum[threadIdx.x] += ssum[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smax[0];
    part[2 * blockIdx.x + 1] = ssum[0];
  }
}

__global__ void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                              double* __restrict__ part) {
  __shared__ double ssum[256];
  double sm = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    sm += a[t] * b[t];
  ssum[threadIdx.x] = sm;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) ssum[threadIdx.x] += ssum[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = 0.0;
    part[2 * blockIdx.x + 1] = ssum[0];
  }
}

__global__ void k_reduce_final(const double* __restrict__ part, int nb, double* __restrict__ out,
                               double* host_out, double* seq) {
  __shared__ double smax[256], ssum[256];
  double mx = 0.0, sm = 0.0;
  for (int t = threadIdx.x; t < nb; t += blockDim.x) {
    mx = nanmax(mx, part[2 * t]);
    sm += part[2 * t + 1];
  }
  smax[threadIdx.x] = mx;
  ssum[threadIdx.x] = sm;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      smax[threadIdx.x] = nanmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      ssum[threadIdx.x] += ssum[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smax[0];
    out[1] = ssum[0];
    // straight to pinned host memory; the sequence number (counted on the
    // device, so a replayed graph still numbers its reductions) goes last
    const double q = seq[0] + 1.0;
    seq[0] = q;
    host_out[0] = smax[0];
    host_out[1] = ssum[0];
    __threadfence_system();
    host_out[2] = q;
    __threadfence_system();
  }
}

// y = S x (or S^T x) for a 9-plane stencil S on the fine grid
__global__ void k_stencil_apply(const double* __restrict__ S, const double* __restrict__ x,
                                double* __restrict__ y, int N, int transpose) {
  const int s = N + 1;
  const int64_t n = (int64_t)s * s;
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = (int)(k % s), j = (int)(k / s);
  double acc = 0.0;
  for (int p = 0; p < 9; ++p) {
    const int dx = p % 3 - 1, dy = p / 3 - 1;
    const int ii = i + dx, jj = j + dy;
    if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
    const int64_t kk = ii + (int64_t)jj * s;
    // row k, column kk uses plane p at k; the transpose reads row kk's
    // coefficient of column k, i.e. plane (8 - p) at kk
    const double a = transpose ? S[(8 - p) * n + kk] : S[p * n + k];
    if (a != 0.0) acc += a * x[kk];
  }
  y[k] = acc;
}

// per-block (max |v|, sum v^2) of a block of 256 threads into part[2 b], part[2 b + 1]
__device__ inline void block_pair(double mx, double sm, double* __restrict__ part) {
  __shared__ double smax[256], ssum[256];
  smax[threadIdx.x] = mx;
  ssum[threadIdx.x] = sm;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      smax[threadIdx.x] = nanmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      ssum[threadIdx.x] += ssum[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smax[0];
    part[2 * blockIdx.x + 1] = ssum[0];
  }
}

// F = M f + G g on the box of active nodes (section 2, the discrete load):
// a row whose four cells are interior has the constant Q1 mass stencil
// h^2/36 [1 4 1; 4 16 4; 1 4 1] and no boundary term; other rows read their
// stored M and G planes.  Also reduces (max |F|, sum F^2).
__global__ void k_rhs(const double* __restrict__ M, const double* __restrict__ G,
                      const uint8_t* __restrict__ fl, const double* __restrict__ f,
                      const double* __restrict__ g, double* __restrict__ F, int N, double hh36, int i0,
                      int j0, int ni, int nj, double* __restrict__ part) {
  const int s = N + 1;
  const int64_t n = (int64_t)s * s;
  const int64_t tot = (int64_t)ni * nj;
  double mx = 0.0, sm = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = i0 + (int)(t % ni), j = j0 + (int)(t / ni);
    const int64_t k = i + (int64_t)j * s;
    const uint8_t fk = fl[k];
    double acc = 0.0;
    if (!(fk & kFlagActive)) {
      F[k] = 0.0;
      continue;
    }
    if (!(fk & kFlagStored)) {
      const double corners = (f[k - s - 1] + f[k - s + 1]) + (f[k + s - 1] + f[k + s + 1]);
      const double edges = (f[k - s] + f[k + s]) + (f[k - 1] + f[k + 1]);
      acc = hh36 * (16.0 * f[k] + 4.0 * edges + corners);
    } else {
      for (int p = 0; p < 9; ++p) {
        const int ii = i + p % 3 - 1, jj = j + p / 3 - 1;
        if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
        const int64_t kk = ii + (int64_t)jj * s;
        const double m = M[p * n + k], gg = G[p * n + k];
        if (m != 0.0) acc += m * f[kk];
        if (gg != 0.0) acc += gg * g[kk];
      }
    }
    F[k] = acc;
    mx = nanmax(mx, fabs(acc));
    sm += acc * acc;
  }
  block_pair(mx, sm, part);
}

// Outer step of the mixed-precision solve, on the box of active nodes:
// u_new = u + e (e: the float correction, null for none), r = F - A u_new in
// float64, the float copy of r as the next inner right-hand side, a zero
// float start iterate for the next inner cycle, and (max |r|, sum r^2).
// u_new goes to a second buffer, so every thread reads the old u.
__global__ void k_outer(LevelView<double> v, const double* __restrict__ F, const double* __restrict__ u,
                        const float* __restrict__ e, double* __restrict__ u_out, float* __restrict__ r32,
                        float* __restrict__ z32, int i0, int j0, int ni, int nj, double* __restrict__ part) {
  const int64_t tot = (int64_t)ni * nj;
  const int s = v.s;
  double mx = 0.0, sm = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = i0 + (int)(t % ni), j = j0 + (int)(t / ni);
    const int64_t k = i + (int64_t)j * s;
    const uint8_t f = v.fl[k];
    if (!(f & kFlagActive)) continue;
    auto un = [&](int64_t q) { return e ? u[q] + (double)e[q] : u[q]; };
    const double uk = un(k);
    double ax;
    if (f & kFlagStored) {
      const double* A = v.A;
      const int64_t n = v.n;
      ax = A[4 * n + k] * uk;
      const bool w = i > 0, ea = i < v.N, so = j > 0, no = j < v.N;
      if (so) {
        if (w) ax += A[k] * un(k - s - 1);
        ax += A[n + k] * un(k - s);
        if (ea) ax += A[2 * n + k] * un(k - s + 1);
      }
      if (w) ax += A[3 * n + k] * un(k - 1);
      if (ea) ax += A[5 * n + k] * un(k + 1);
      if (no) {
        if (w) ax += A[6 * n + k] * un(k + s - 1);
        ax += A[7 * n + k] * un(k + s);
        if (ea) ax += A[8 * n + k] * un(k + s + 1);
      }
    } else {
      const double nb = (un(k - s - 1) + un(k - s) + un(k - s + 1)) + (un(k - 1) + un(k + 1)) +
                        (un(k + s - 1) + un(k + s) + un(k + s + 1));
      ax = 8.0 / 3.0 * uk - nb / 3.0;
    }
    const double r = F[k] - ax;
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

void launch_rhs(mgfem_ctx* c, const double* f, const double* g, double* F) {
  const Level& L = c->lv[0];
  const int ni = L.bbox[1] - L.bbox[0] + 1, nj = L.bbox[3] - L.bbox[2] + 1;
  const int64_t tot = (int64_t)ni * nj;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (tot + 255) / 256));
  hipLaunchKernelGGL(k_rhs, dim3(nb), dim3(256), 0, c->s, c->M, c->G, L.flags, f, g, F, c->N,
                     c->h * c->h / 36.0, L.bbox[0], L.bbox[2], ni, nj, c->red_partial);
  c->red_seq += 1.0;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, c->s, c->red_partial, nb, c->red_out, c->red_host,
                     c->red_seq_dev);
}

void launch_outer(mgfem_ctx* c, const double* u, const float* e, double* u_out, float* r32, float* z32) {
  Level& L = c->lv[0];
  LevelView<double> v{L.A, L.flags, nullptr, nullptr, nullptr, L.N, L.stride, L.n};
  const int ni = L.bbox[1] - L.bbox[0] + 1, nj = L.bbox[3] - L.bbox[2] + 1;
  const int64_t tot = (int64_t)ni * nj;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (tot + 255) / 256));
  hipLaunchKernelGGL(k_outer, dim3(nb), dim3(256), 0, c->s, v, (const double*)L.b, u, e, u_out, r32, z32,
                     L.bbox[0], L.bbox[2], ni, nj, c->red_partial);
  c->red_seq += 1.0;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, c->s, c->red_partial, nb, c->red_out, c->red_host,
                     c->red_seq_dev);
}

void launch_stencil_apply(mgfem_ctx* c, const double* planes, const double* x, double* y, bool transpose) {
  const int64_t n = c->lv[0].n;
  hipLaunchKernelGGL(k_stencil_apply, dim3(nblk(n, 256)), dim3(256), 0, c->s, planes, x, y, c->N,
                     transpose ? 1 : 0);
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
  const int64_t tot = (int64_t)ni * nj;
  const int nb = (int)std::min<int64_t>(kRedBlocks, (tot + 255) / 256);
  hipLaunchKernelGGL(k_resnorm_partial, dim3(nb), dim3(256), 0, c->s, v, F, r_out, L.bbox[0],
                     L.bbox[2], ni, nj, c->red_partial);
  c->red_seq += 1.0;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, c->s, c->red_partial, nb, c->red_out, c->red_host,
                     c->red_seq_dev);
}

void launch_dot_reduce(mgfem_ctx* c, const double* a, const double* b) {
  const int64_t n = c->lv[0].n;
  const int nb = (int)std::min<int64_t>(kRedBlocks, (n + 255) / 256);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(256), 0, c->s, a, b, n, c->red_partial);
  c->red_seq += 1.0;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, c->s, c->red_partial, nb, c->red_out, c->red_host,
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
