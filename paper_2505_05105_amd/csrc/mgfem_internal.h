// Internal declarations of the gfx950 ghost-FEM multigrid library.
//
// Data layout per grid level l (N_l cells per side, n_l = (N_l+1)^2 nodes,
// node (i,j) at flat index i + j (N_l+1)):
//   A     9 planes of n_l doubles (structure of arrays); plane p = (di+1) +
//         3 (dj+1) is the coefficient of node (i+di, j+dj) in row (i,j).
//   flags one byte per node: bit 0 active (non-zero diagonal), bit 1 the row
//         must be read from A (otherwise it is the constant interior Q1
//         stencil 8/3, -1/3), bit 2 vertex of a cut cell (extra smoothing).
//   x, b, r  iterate, right-hand side and residual (and float copies for the
//         mixed-precision inner cycles).
//   cut lists  node indices of the extra-smoothing set, one list per colour
//         c = (i mod 2) + 2 (j mod 2), ascending.
// Level 0 also holds the mass and boundary-load stencils (M, G), the snapped
// level set, cell types and lambda_K.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mgfem.h"

namespace mgfem {

constexpr int kFlagActive = 1;
constexpr int kFlagStored = 2;
constexpr int kFlagCut = 4;

// cell type codes
constexpr int kExternal = 0, kTriangle = 1, kQuad = 2, kPentagon = 3, kInternal = 4,
              kSaddleSplit = 5, kSaddleHex = 6;

struct Level {
  int N = 0;
  int stride = 0;  // N + 1
  int64_t n = 0;   // (N+1)^2
  double* A = nullptr;
  float* A32 = nullptr;
  uint8_t* flags = nullptr;
  uint8_t* cellcut = nullptr;  // N*N, 1 on cut cells of this level
  double *x = nullptr, *b = nullptr, *r = nullptr;
  float *x32 = nullptr, *b32 = nullptr, *r32 = nullptr;
  int* cut_list = nullptr;  // concatenated colour lists
  int cut_off[5] = {0, 0, 0, 0, 0};
  int bbox[4] = {1, 0, 1, 0};  // i_lo, i_hi, j_lo, j_hi of active nodes (inclusive)
  bool empty() const { return bbox[0] > bbox[1]; }
};

struct Stats {
  unsigned long long counts[7];
  unsigned long long snapped;
  unsigned long long active;
  unsigned long long min_theta_bits;   // float64 bits of the minimum (positive) theta
  unsigned long long max_lambda_bits;  // float64 bits of the maximum lambda
  int coarse_status;                   // 0 ok, 1 singular
  int coarse_n;
};

}  // namespace mgfem

struct mgfem_ctx {
  mgfem_params p{};
  hipStream_t s = nullptr;
  int N = 0;
  double h = 0.0;
  std::vector<mgfem::Level> lv;
  // level-0 extras
  double* psi = nullptr;
  uint8_t* cell_type = nullptr;
  double* cell_lambda = nullptr;
  double* M = nullptr;
  double* G = nullptr;
  double* F = nullptr;
  double* F64tmp = nullptr;  // outer residual / scratch on level 0
  double* zero = nullptr;    // all-zero vector of level 0
  double* lam = nullptr;     // adjoint state when the caller passes none
  // coarsest exact solve
  double* coarse_L = nullptr;  // cn x cn lower Cholesky factor
  int* coarse_idx = nullptr;   // cn node indices
  int coarse_n = 0;
  // reductions
  double* red_partial = nullptr;  // 2 * kRedBlocks
  double* red_out = nullptr;      // 2 doubles on device
  double* red_host = nullptr;     // pinned, 2 doubles
  mgfem::Stats* stats = nullptr;  // device
  mgfem_info info{};
  std::vector<void*> allocs;
  std::string last_error;
  bool batched_member = false;
};

namespace mgfem {

constexpr int kRedBlocks = 1024;

// memory helpers (record the allocation on the context)
hipError_t ctx_alloc(mgfem_ctx* c, void** p, size_t bytes);
template <class T>
hipError_t ctx_alloc_t(mgfem_ctx* c, T** p, size_t count) {
  return ctx_alloc(c, reinterpret_cast<void**>(p), count * sizeof(T));
}

// setup stages (geometry.hip, hierarchy.hip)
int setup_geometry(mgfem_ctx* c, const double* psi_in);
int setup_hierarchy(mgfem_ctx* c);

// solve stages (cycle.hip)
void launch_rhs(mgfem_ctx* c, const double* f, const double* g, double* F);
void launch_stencil_apply(mgfem_ctx* c, const double* planes, const double* x, double* y, bool transpose);
void launch_mask_inactive(mgfem_ctx* c, double* u);
void launch_residual_norm(mgfem_ctx* c, const double* F, const double* u, double* r_out);
void launch_dot_reduce(mgfem_ctx* c, const double* a, const double* b);
void launch_zero(mgfem_ctx* c, double* p, int64_t n);
void launch_copy(mgfem_ctx* c, double* dst, const double* src, int64_t n);
void launch_axpy_active(mgfem_ctx* c, double* u, const float* e);
void launch_cast_to_float(mgfem_ctx* c, float* dst, const double* src, int64_t n);
void launch_sub_active(mgfem_ctx* c, double* d, const double* a, const double* b);
void launch_zero_f(mgfem_ctx* c, float* p, int64_t n);
void launch_u8_to_f64(mgfem_ctx* c, const uint8_t* s, double* d, int64_t n);

struct CycleOpts {
  bool reverse = false;  // transposed cycle (adjoint)
  bool fp32 = false;     // float inner cycle
};
// one cycle on level 0 with x = lv[0].x*, b = lv[0].b* (pointers set by the caller)
void run_cycle(mgfem_ctx* c, const CycleOpts& o);
void smooth_level(mgfem_ctx* c, int l, bool reverse, bool fp32);

}  // namespace mgfem

#define MGFEM_HIP_TRY(expr)                                                   \
  do {                                                                        \
    hipError_t _e = (expr);                                                   \
    if (_e != hipSuccess) {                                                   \
      c->last_error = std::string(#expr) + ": " + hipGetErrorString(_e);      \
      return _e == hipErrorOutOfMemory ? MGFEM_ERR_OOM : MGFEM_ERR_HIP;       \
    }                                                                         \
  } while (0)
