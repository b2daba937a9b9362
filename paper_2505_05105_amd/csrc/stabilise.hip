// Vector kernels of the Lanczos iteration that finds the global stabilisation
// constant (section 5.2): C = max Lambda of K v = Lambda S v.  The driver is
// in api.hip; these are the level-0 vector updates it needs between the
// operator applications (K from the gathered cut-vertex rows, S and S^-1 from
// the stiffness context's residual kernel and multigrid solve).
#include "mgfem_internal.h"

namespace mgfem {
namespace {

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

// splitmix64 of the node index: a fixed start vector in [-1/2, 1/2) on the
// active nodes (any vector with a component along the top eigenvector serves)
__global__ void k_start(const uint8_t* __restrict__ fl, double* __restrict__ x, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint64_t z = (uint64_t)k + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  const double v = (double)(z >> 11) * 0x1.0p-53 - 0.5;
  x[k] = (fl[k] & kFlagActive) ? v : 0.0;
}

__global__ void k_ones(const uint8_t* __restrict__ fl, double* __restrict__ x, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) x[k] = (fl[k] & kFlagActive) ? 1.0 : 0.0;
}

// w = w - a q - b qp
__global__ void k_lanczos(double* __restrict__ w, const double* __restrict__ q, const double* __restrict__ qp,
                          double a, double b, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) w[k] = (w[k] - a * q[k]) - b * qp[k];
}

__global__ void k_shift(const uint8_t* __restrict__ fl, double* __restrict__ w, double v, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n && (fl[k] & kFlagActive)) w[k] -= v;
}

__global__ void k_scale(double* __restrict__ d, const double* __restrict__ s, double f, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) d[k] = s[k] * f;
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) y[k] += a * x[k];
}

}  // namespace

void launch_start_vector(mgfem_ctx* c, double* x) {
  const int64_t n = c->lv[0].n;
  hipLaunchKernelGGL(k_start, dim3(nb256(n)), dim3(256), 0, c->s, c->lv[0].flags, x, n);
}
void launch_active_ones(mgfem_ctx* c, double* x) {
  const int64_t n = c->lv[0].n;
  hipLaunchKernelGGL(k_ones, dim3(nb256(n)), dim3(256), 0, c->s, c->lv[0].flags, x, n);
}
void launch_lanczos_update(mgfem_ctx* c, double* w, const double* q, const double* qp, double a, double b) {
  const int64_t n = c->lv[0].n;
  hipLaunchKernelGGL(k_lanczos, dim3(nb256(n)), dim3(256), 0, c->s, w, q, qp, a, b, n);
}
void launch_shift_active(mgfem_ctx* c, double* w, double v) {
  const int64_t n = c->lv[0].n;
  hipLaunchKernelGGL(k_shift, dim3(nb256(n)), dim3(256), 0, c->s, c->lv[0].flags, w, v, n);
}
void launch_scale(mgfem_ctx* c, double* dst, const double* src, double f) {
  const int64_t n = c->lv[0].n;
  hipLaunchKernelGGL(k_scale, dim3(nb256(n)), dim3(256), 0, c->s, dst, src, f, n);
}
void launch_axpy(mgfem_ctx* c, double* y, const double* x, double a) {
  const int64_t n = c->lv[0].n;
  hipLaunchKernelGGL(k_axpy, dim3(nb256(n)), dim3(256), 0, c->s, y, x, a, n);
}

}  // namespace mgfem
