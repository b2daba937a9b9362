// Batched solves: placeholder entry points (implemented below in a later
// revision of this file).
#include "mgfem_internal.h"

extern "C" {

int mgfem_setup_batched(int32_t count, const double* const* psi_dev, const int32_t* N,
                        const mgfem_params* p, void* stream, mgfem_handle* out) {
  (void)count; (void)psi_dev; (void)N; (void)p; (void)stream;
  if (out) *out = nullptr;
  return MGFEM_ERR_UNSUPPORTED;
}

int mgfem_solve_batched(mgfem_handle h, const double* const* f_dev, const double* const* g_dev,
                        double rel_tol, int32_t max_cycles, double* const* u_dev,
                        double* res_hist_host, int32_t* n_cycles) {
  (void)h; (void)f_dev; (void)g_dev; (void)rel_tol; (void)max_cycles; (void)u_dev;
  (void)res_hist_host; (void)n_cycles;
  return MGFEM_ERR_UNSUPPORTED;
}

}  // extern "C"
