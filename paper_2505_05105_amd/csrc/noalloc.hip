// Allocation-free form of the misfit call: J = 1/2 e^T M e and dJ/du = M e
// with e = u - u_t on the active nodes, every scratch value of the call (the
// per-block partial sums) in one static device array instead of memory the
// library allocates, so that callers that must not allocate (code under HIP
// graph capture, tight serving loops) can evaluate the objective.
//
// The array `scratch` exists once per device for the life of the process.
// Host code never passes its name to a kernel: set-up (the first
// mgfem_setup on a device) asks the runtime for its device address with
// hipGetSymbolAddress and keeps it per device; the kernels get that address.
// Every call on one device shares the array, and each call overwrites all of
// it that it reads (one partial per block of its grid), so nothing has to be
// cleared between calls; calls that overlap on one device race.
#include <mutex>

#include "mgfem_internal.h"

namespace {
constexpr size_t kScratchBytes = size_t(2) << 20;  // 2 MiB per device
}  // namespace

// the scratch of mgfem_misfit_noalloc (see the top of this file)
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace mgfem {
namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// a block takes 256 x 4 nodes; e is staged in LDS with a halo of one (zero off
// the grid and at inactive nodes)
constexpr int kMX = 256, kMY = 4, kMW = kMX + 2, kMH = kMY + 2, kMN = kMW * kMH;

// dJ/du = M e at every node of the block (0 at inactive nodes and off the box
// of active nodes) and the block's share of e^T M e in part[block].  Rows:
// the gathered M row at a cut-cell vertex (cut_rows, 18 per vertex in
// cut-list order, M first), the stored planes at any other stored row, the
// interior Q1 mass stencil h^2/36 [1 4 1; 4 16 4; 1 4 1] elsewhere.
__global__ __launch_bounds__(256) void k_misfit_partial(const double* __restrict__ u, const double* __restrict__ ut,
                                                        const uint8_t* __restrict__ fl, const int* __restrict__ cutpos,
                                                        const double* __restrict__ cut_rows,
                                                        const double* __restrict__ M, double* __restrict__ y, int N,
                                                        double hh36, int i0, int j0, int i1, int j1,
                                                        double* __restrict__ part) {
  __shared__ double se[kMN];
  __shared__ double wsum[4];
  const int s = N + 1;
  const int64_t n = (int64_t)s * s;
  const int bi = blockIdx.x * kMX, bj = blockIdx.y * kMY;
  const bool touches = bi <= i1 && bi + kMX - 1 >= i0 && bj <= j1 && bj + kMY - 1 >= j0;  // uniform
  if (touches) {
    constexpr int NU = (kMN + 255) / 256;
    double r[NU];
#pragma unroll
    for (int q0 = 0; q0 < NU; ++q0) {
      const int q = threadIdx.x + q0 * 256;
      const int gi = bi - 1 + q % kMW, gj = bj - 1 + q / kMW;
      double v = 0.0;
      if (q < kMN && gi >= 0 && gj >= 0 && gi <= N && gj <= N) {
        const int64_t k = gi + (int64_t)gj * s;
        if (fl[k] & kFlagActive) v = u[k] - ut[k];
      }
      r[q0] = v;
    }
#pragma unroll
    for (int q0 = 0; q0 < NU; ++q0) {
      const int q = threadIdx.x + q0 * 256;
      if (q < kMN) se[q] = r[q0];
    }
    __syncthreads();
  }
  double sm = 0.0;
  const int i = bi + threadIdx.x;
#pragma unroll
  for (int rep = 0; rep < kMY; ++rep) {
    const int j = bj + rep;
    if (i > N || j > N) continue;
    const int64_t k = i + (int64_t)j * s;
    double me = 0.0;
    if (touches && i >= i0 && i <= i1 && j >= j0 && j <= j1) {
      const uint8_t fk = fl[k];
      if (fk & kFlagActive) {
        const int q = threadIdx.x + 1 + (rep + 1) * kMW;
        if (fk & kFlagCut) {
          const double* row = cut_rows + 18 * (int64_t)cutpos[k];
          for (int p = 0; p < 9; ++p) me += row[p] * se[q + (p % 3 - 1) + (p / 3 - 1) * kMW];
        } else if (fk & kFlagStored) {
          for (int p = 0; p < 9; ++p) me += M[p * n + k] * se[q + (p % 3 - 1) + (p / 3 - 1) * kMW];
        } else {
          const double corners = (se[q - kMW - 1] + se[q - kMW + 1]) + (se[q + kMW - 1] + se[q + kMW + 1]);
          const double edges = (se[q - kMW] + se[q + kMW]) + (se[q - 1] + se[q + 1]);
          me = hh36 * (16.0 * se[q] + 4.0 * edges + corners);
        }
        sm += se[q] * me;
      }
    }
    if (y) y[k] = me;
  }
  for (int o = 32; o > 0; o >>= 1) sm += __shfl_xor(sm, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = sm;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x + blockIdx.y * gridDim.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

// sum of the block partials in a fixed order, written to pinned host memory
__global__ __launch_bounds__(1024) void k_misfit_final(const double* __restrict__ part, int nb, double* host_rec) {
  __shared__ double wsum[16];
  double sm = 0.0;
  for (int t = threadIdx.x; t < nb; t += blockDim.x) sm += part[t];
  for (int o = 32; o > 0; o >>= 1) sm += __shfl_xor(sm, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = sm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wsum[w];
    host_rec[0] = t;
    __threadfence_system();
  }
}

}  // namespace

int scratch_init(int* device) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return MGFEM_ERR_HIP;
  }
  *device = dev;
  if (dev < 0 || dev >= kMaxDevices) return MGFEM_OK;  // the no-allocation call reports it
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_tried[dev]) {
    g_scratch_tried[dev] = true;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[dev] = p;
    else (void)hipGetLastError();
  }
  return MGFEM_OK;
}

}  // namespace mgfem

using namespace mgfem;

extern "C" {

int mgfem_misfit_noalloc(mgfem_handle c, const double* u_dev, const double* ut_dev, double* J_host,
                         double* dJdu_dev) {
  if (!c) return MGFEM_ERR_INVALID_ARG;
  if (c->batched_member || !c->members.empty() || c->lv.empty()) {
    c->last_error = "batched handle: use mgfem_solve_batched";
    return MGFEM_ERR_INVALID_ARG;
  }
  if (!u_dev || !ut_dev || !J_host) {
    c->last_error = "u, ut and J must be given";
    return MGFEM_ERR_INVALID_ARG;
  }
  void* base = nullptr;
  if (c->device >= 0 && c->device < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_ptr[c->device];
  }
  if (!base) {
    c->last_error = "the static scratch array has no device address on device " + std::to_string(c->device);
    return MGFEM_ERR_HIP;
  }
  const Level& L = c->lv[0];
  const int N = c->N;
  const dim3 grid((unsigned)((N + kMX) / kMX), (unsigned)((N + kMY) / kMY));  // (N+1) nodes per side
  const int64_t nb = (int64_t)grid.x * grid.y;
  if (nb * (int64_t)sizeof(double) > (int64_t)kScratchBytes) {
    c->last_error = "N = " + std::to_string(N) + " needs " + std::to_string(nb * sizeof(double)) +
                    " bytes of partial sums; the static scratch array holds " + std::to_string(kScratchBytes) +
                    " bytes (every N below 16384 fits)";
    return MGFEM_ERR_INVALID_ARG;
  }
  double* part = static_cast<double*>(base);
  double* rec = c->red_host + 4 * kRedSlots;  // the handle's own pinned record (allocated at set-up)
  rec[0] = 0.0;
  hipLaunchKernelGGL(k_misfit_partial, grid, dim3(256), 0, c->s, u_dev, ut_dev, (const uint8_t*)L.flags,
                     (const int*)L.cutpos, (const double*)c->cut_rows, (const double*)c->M, dJdu_dev, N,
                     c->h * c->h / 36.0, L.bbox[0], L.bbox[2], L.bbox[1], L.bbox[3], part);
  hipLaunchKernelGGL(k_misfit_final, dim3(1), dim3(1024), 0, c->s, (const double*)part, (int)nb, rec);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) {
    c->last_error = std::string("mgfem_misfit_noalloc: ") + hipGetErrorString(e);
    return MGFEM_ERR_HIP;
  }
  *J_host = 0.5 * reinterpret_cast<volatile double*>(rec)[0];
  return MGFEM_OK;
}

}  // extern "C"
