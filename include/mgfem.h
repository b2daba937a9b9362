/*
 * mgfem.h -- C ABI of the MI355X (gfx950) multigrid solver for the nodal
 * ghost finite-element discretisation of the Poisson problem on a domain
 * given by a level set (Dilip & Coco, "Multigrid methods for the ghost finite
 * element approximation of elliptic problems", arXiv 2505.05105).
 *
 * Problem (section 2): -lap u = f in Omega = {psi < 0}, u = g on its boundary
 * (or u = g_D on a Dirichlet part and n . grad u = g_N on a Neumann part,
 * mgfem_setup_mixed_bc), discretised with Q1 elements on the active cells of
 * a uniform N x N grid over a box, Dirichlet data imposed weakly by Nitsche's
 * method (eqs. disc_bil_form, disc_rhs) with the cell-wise stabilisation
 * lambda_K = gamma C(K) or one global lambda (section 5.2), after snapping
 * back to grid (section 2).
 * Solver (sections 3 and 5): Gauss-Seidel smoothing in four colours plus eta
 * extra sweeps on the vertices of cut cells, restriction by the transposed
 * bilinear prolongation, Galerkin (or re-discretised) coarse operators, exact
 * solve on the coarsest grid, V- or W-cycles or the two-grid scheme.
 *
 * Conventions shared by every call:
 *  - Grid arrays are float64 arrays in device memory of length (N+1)^2; node
 *    (i, j) at (x_lo + i h, y_lo + j h), h = (x_hi - x_lo)/N, has flat index
 *    k = i + j (N+1) (the single index of section 5.1).  Cell (i, j) has flat
 *    index i + j N.
 *  - The caller owns every array it passes; the library never frees or keeps
 *    a caller pointer after a call returns.  The library owns the handle and
 *    all of its workspace (hierarchy, stencils, lists).
 *  - Work is enqueued on the stream given to setup (a hipStream_t passed as
 *    void*; NULL is the default stream).  Calls that return host results
 *    synchronise that stream before they return.
 *  - Every call returns an mgfem_status code and never throws.  On an error
 *    the outputs are unspecified, except MGFEM_ERR_NOT_CONVERGED: then u and
 *    the residual history are valid for the cycles that were run.
 *  - Nodes that are not vertices of an active cell ("inactive") hold 0 in
 *    every output array.
 *  - A handle may be used by one host thread at a time.
 */
#ifndef MGFEM_H
#define MGFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgfem_ctx* mgfem_handle;

enum mgfem_status {
  MGFEM_OK = 0,
  MGFEM_ERR_INVALID_ARG = 1,     /* bad size, pointer or parameter */
  MGFEM_ERR_OOM = 2,             /* device allocation failed */
  MGFEM_ERR_HIP = 3,             /* a HIP runtime call failed */
  MGFEM_ERR_NOT_CONVERGED = 4,   /* max_cycles reached above the tolerance */
  MGFEM_ERR_DIVERGED = 5,        /* non-finite residual, or growth over 3 cycles */
  MGFEM_ERR_SINGULAR_COARSE = 6, /* non-positive pivot in the coarsest Cholesky */
  MGFEM_ERR_EMPTY_DOMAIN = 7,    /* no node with psi < 0 after snapping */
  MGFEM_ERR_UNSUPPORTED = 8      /* option not supported by the library */
};

/* Stabilisation rule for lambda_K = gamma C(K) (section 5.2). */
enum mgfem_stab {
  MGFEM_STAB_PAPER = 0,     /* closed forms: eq. c_triangle, the quadrilateral
                               formula, eq. c_pentagon for pentagons */
  MGFEM_STAB_LOCAL_EIG = 1, /* max eigenvalue of the local 4x4 generalised
                               eigenproblem of section 5.2 */
  MGFEM_STAB_FIXED = 2,     /* lambda_K = lambda_fixed on every cut cell */
  MGFEM_STAB_GLOBAL = 3     /* one lambda = gamma C on every cut cell, C the largest
                               eigenvalue of the global generalised eigenproblem
                               K v = Lambda S v of section 5.2 (K over Gamma_D, S the
                               stiffness over Omega), found at setup by Lanczos
                               iterations with multigrid solves for S; not with
                               MGFEM_COARSE_REDISCRETISED */
};

enum mgfem_precision {
  MGFEM_PREC_FP64 = 0,  /* every cycle in float64 */
  MGFEM_PREC_MIXED = 1  /* float32 cycles inside float64 defect correction;
                           float64 outer residual, geometry and coarsest solve */
};

enum mgfem_cycle {
  MGFEM_CYCLE_V = 1,        /* gamma* = 1 (section 3.2) */
  MGFEM_CYCLE_W = 2,        /* gamma* = 2 (section 3.2) */
  MGFEM_CYCLE_TWO_GRID = 3  /* two-grid correction scheme (Algorithm 1 of section 3.1):
                               the first coarse problem is solved by coarse_cycles
                               V-cycles from zero, which reduce its error far below
                               float64 rounding (an exact solve in effect); the
                               levels below serve that inner solve only */
};

/* coarse-level operators (section 4.3 and section 5) */
enum mgfem_coarse_op {
  MGFEM_COARSE_GALERKIN = 0,     /* A_{2h} = R A_h P (eq. galerkin) */
  MGFEM_COARSE_REDISCRETISED = 1 /* every coarse level assembled from scratch on its own grid:
                                    psi injected at the coarse nodes (coarse node (I, J) is
                                    fine node (2I, 2J)), snapped, classified, stabilised and
                                    assembled with the coarse cell size; its extra-smoothing
                                    set is the vertices of its own cut cells */
};

#define MGFEM_SOLVE_WARM_START 1u /* start from the u passed in, not from 0 */

typedef struct {
  int32_t stab_rule;    /* enum mgfem_stab, default MGFEM_STAB_PAPER */
  double gamma;         /* lambda_K = gamma C(K); must exceed 1 (section 4.4); default 2 */
  double lambda_fixed;  /* used by MGFEM_STAB_FIXED only */
  double snap_alpha;    /* snapping threshold h^alpha (section 2); default 1.75 */
  int32_t nu1, nu2;     /* pre/post smoothing steps; default 2, 1 */
  int32_t eta;          /* extra cut-cell sweeps per smoothing step; default 4 */
  int32_t coarsest_n;   /* cells per side of the coarsest grid; default 4 */
  int32_t precision;    /* enum mgfem_precision, default MGFEM_PREC_FP64 */
  int32_t cycle;        /* enum mgfem_cycle, default MGFEM_CYCLE_V */
  double x_lo, y_lo, x_hi, y_hi; /* square box; default [-1, 1]^2 */
  int32_t coarse_cycles; /* MGFEM_CYCLE_TWO_GRID: V-cycles of the coarse solve (1..1000); default 40 */
  int32_t coarse_op;     /* enum mgfem_coarse_op, default MGFEM_COARSE_GALERKIN */
  int32_t inner_cycles;  /* MGFEM_PREC_MIXED: float32 cycles per float64 defect-correction
                            step (1..16; the first starts from zero, the others continue
                            from it); default 3.  With rel_tol > 0 a step runs fewer
                            where the factor per float32 cycle of an earlier step says
                            fewer reach the tolerance (environment MGFEM_FIXED_INNER=1
                            keeps the full count; mgfem_step_cycles reports the counts).
                            The residual history and max_cycles count the
                            defect-correction steps */
} mgfem_params;

typedef struct {
  int32_t N;                 /* cells per side of the finest grid */
  int32_t n_levels;          /* grids in the hierarchy, finest to coarsest */
  int64_t n_active;          /* active fine nodes (degrees of freedom) */
  int64_t n_cells_by_type[7];/* external, triangle, quadrilateral, pentagon,
                                internal, saddle split, saddle hexagon */
  int64_t n_snapped;         /* nodes whose psi was set to 0 by snapping */
  int64_t n_cut_vertices;    /* fine nodes in the extra-smoothing set */
  int32_t coarse_n;          /* unknowns of the coarsest exact solve */
  double min_theta;          /* smallest cut fraction on a cut edge */
  double max_lambda;         /* largest lambda_K */
  double setup_ms;           /* device time of the last setup */
  double global_C;           /* MGFEM_STAB_GLOBAL: C of the global eigenproblem, else 0 */
  int32_t global_iters;      /* MGFEM_STAB_GLOBAL: Lanczos steps taken, else 0 */
} mgfem_info;

/* Fill *p with the defaults listed above. */
int mgfem_default_params(mgfem_params* p);

/*
 * Build the solver for one level set.
 *  psi_dev : device, (N+1)^2 float64 nodal values of psi (read only).
 *  N       : cells per side; must be coarsest_n times a power of two, >= 2 coarsest_n.
 *  p       : parameters (NULL for the defaults).
 *  stream  : hipStream_t as void* (NULL = default stream).
 *  out     : receives the handle; release it with mgfem_destroy.
 * Runs snapping, cell classification and cut geometry, C(K) and lambda_K,
 * the fine stencils of A, M and G, the Galerkin hierarchy, the cut-vertex
 * lists and the coarsest Cholesky factor, all on the device.
 * Errors: INVALID_ARG, OOM, HIP, EMPTY_DOMAIN, SINGULAR_COARSE.
 */
int mgfem_setup(const double* psi_dev, int32_t N, const mgfem_params* p, void* stream,
                mgfem_handle* out);

/*
 * Mixed Dirichlet/Neumann boundaries (section 2: -lap u = f, u = g_D on
 * Gamma_D, n . grad u = g_N on Gamma_N; eqs. disc_bil_form and disc_rhs).
 * As mgfem_setup, plus
 *  chi_dev : device, (N+1)^2 float64 nodal indicator of the Neumann part
 *            (read only; NULL: the whole boundary is Dirichlet, as mgfem_setup).
 * An interface segment of a cut cell belongs to Gamma_N when the bilinear
 * interpolant of chi at the segment's midpoint is > 0, else to Gamma_D (the
 * paper leaves this assignment open).  Penalty and Nitsche terms, and C(K),
 * use the Dirichlet segments only; a cell with no Dirichlet segment has
 * lambda_K = 0.  The Neumann segments give GN_ij = int_{Gamma_N} phi_i phi_j,
 * the load matrix of g_N.  Coarse levels assembled on their own grids
 * (MGFEM_COARSE_REDISCRETISED) take chi at their nodes like psi.
 * Solve such a handle with mgfem_solve_mixed_bc (mgfem_solve: g_N = 0).
 * Errors: as mgfem_setup; INVALID_ARG when no segment is a Dirichlet segment
 * (the problem would be singular: constants solve the homogeneous one).
 */
int mgfem_setup_mixed_bc(const double* psi_dev, const double* chi_dev, int32_t N, const mgfem_params* p,
                         void* stream, mgfem_handle* out);

/*
 * Solve A u = F with F = M f + G g (Q1 interpolants of f and g; F follows
 * eq. disc_rhs) by repeated cycles until ||F - A u||_inf <= rel_tol ||F||_inf.
 *  f_dev, g_dev  : device (N+1)^2 float64 nodal source and Dirichlet data
 *                  (g is read on the vertices of cut cells only).
 *  rel_tol       : relative l-infinity residual tolerance (0 or less: run
 *                  exactly max_cycles cycles).
 *  max_cycles    : >= 0.
 *  flags         : MGFEM_SOLVE_WARM_START to start from the incoming u_dev.
 *  u_dev         : device (N+1)^2 float64, receives the solution.
 *  res_hist_host : host, max_cycles+1 float64 or NULL; entry m receives
 *                  ||F - A u_m||_inf (entry 0 for the start), section 3.1.
 *  n_cycles      : host, receives the number of cycles run (may be NULL).
 * In mixed precision one cycle is one float64 outer defect-correction step
 * around up to params.inner_cycles float32 cycles (the first from zero).  Returns
 * OK, NOT_CONVERGED, DIVERGED or an error.
 */
int mgfem_solve(mgfem_handle h, const double* f_dev, const double* g_dev, double rel_tol,
                int32_t max_cycles, uint32_t flags, double* u_dev, double* res_hist_host,
                int32_t* n_cycles);

/*
 * mgfem_solve with Neumann data: F = M f + G g_D + GN g_N (eq. disc_rhs, all
 * three data as Q1 nodal interpolants).
 *  gN_dev : device (N+1)^2 float64 nodal Neumann data, read at the vertices
 *           of cells with a Neumann segment; NULL means g_N = 0.  Ignored for
 *           a handle set up without an indicator.
 * Other arguments, results and errors as mgfem_solve.
 */
int mgfem_solve_mixed_bc(mgfem_handle h, const double* f_dev, const double* gD_dev, const double* gN_dev,
                         double rel_tol, int32_t max_cycles, uint32_t flags, double* u_dev,
                         double* res_hist_host, int32_t* n_cycles);

/*
 * Adjoint of the solve: lam = B_k^T dJ/du with B_k the map F -> u of k cycles,
 * run as k transposed cycles from zero (every smoothing phase in reverse
 * order, nu1 and nu2 swapped); k is fixed by rel_tol/max_cycles as in
 * mgfem_solve.  Then dJ/df = M lam and dJ/dg = G^T lam.
 *  dJdu_dev  : device (N+1)^2 float64.
 *  lam_dev   : device (N+1)^2 float64 or NULL.
 *  dJdf_dev, dJdg_dev : device (N+1)^2 float64 or NULL.
 *  res_hist_host, n_cycles : as in mgfem_solve (history of the adjoint system).
 * Always runs in float64.
 */
int mgfem_adjoint(mgfem_handle h, const double* dJdu_dev, double rel_tol, int32_t max_cycles,
                  double* lam_dev, double* dJdf_dev, double* dJdg_dev, double* res_hist_host,
                  int32_t* n_cycles);

/*
 * Gradient with respect to the Neumann data: dJ/dg_N = GN^T lam = GN lam for
 * the lam of mgfem_adjoint (GN is symmetric; zero for a handle set up
 * without an indicator).
 *  lam_dev, dJdgN_dev : device (N+1)^2 float64.  Synchronises.
 * Errors: INVALID_ARG (NULL pointers, batched handle), HIP.
 */
int mgfem_adjoint_neumann(mgfem_handle h, const double* lam_dev, double* dJdgN_dev);

/*
 * Misfit J = 1/2 (u - u_t)^T M (u - u_t) (nodal interpolants) and
 * dJ/du = M (u - u_t).  J_host: host scalar; dJdu_dev: device (N+1)^2 or NULL.
 */
int mgfem_misfit(mgfem_handle h, const double* u_dev, const double* ut_dev, double* J_host,
                 double* dJdu_dev);

/*
 * mgfem_misfit for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops): same arguments, results and
 * errors, computed by one fused pass whose only scratch (one partial sum per
 * 256 x 4 block of the grid) lives in a static 2 MiB device array of the
 * library instead of memory it allocates.  The call allocates nothing:
 * no hipMalloc, hipFree or allocating library routine.
 *  Limit: (N/256 + 1)(N/4 + 1) partial sums of 8 bytes must fit in 2 MiB
 *         (every N below 16384); a larger N returns INVALID_ARG with the sizes.
 *  Every call on one device shares that array and leaves its partials in
 *  it: calls that overlap on one device (other streams, other host
 *  threads) race.  Synchronises the handle's stream.
 */
int mgfem_misfit_noalloc(mgfem_handle h, const double* u_dev, const double* ut_dev, double* J_host,
                         double* dJdu_dev);

/* Counts and extrema of the setup (fills *info). */
int mgfem_query(mgfem_handle h, mgfem_info* info);

/* What mgfem_export copies out. */
enum mgfem_export_what {
  MGFEM_EXPORT_PSI = 0,        /* snapped psi, (N+1)^2 float64 (level 0 only) */
  MGFEM_EXPORT_CELL_TYPE = 1,  /* cell type codes as float64, N^2 (level 0 only) */
  MGFEM_EXPORT_CELL_LAMBDA = 2,/* lambda_K per cell (0 off cut cells), N^2 float64 */
  MGFEM_EXPORT_A = 3,          /* 9 stencil planes of A_l, 9 (N_l+1)^2 float64;
                                  plane p = (di+1) + 3 (dj+1) holds the coefficient
                                  of node (i+di, j+dj) in row (i, j) */
  MGFEM_EXPORT_M = 4,          /* 9 planes of the mass matrix (level 0 only) */
  MGFEM_EXPORT_G = 5,          /* 9 planes of the boundary-load matrix G (level 0 only) */
  MGFEM_EXPORT_NODE_FLAGS = 6, /* per node, as float64: bit 0 active, bit 1 stored
                                  stencil, bit 2 extra-smoothing vertex */
  MGFEM_EXPORT_RHS = 7,        /* F of the last solve, (N+1)^2 float64 */
  MGFEM_EXPORT_GN = 8          /* 9 planes of the Neumann boundary mass GN (level 0 only;
                                  zero for a handle set up without an indicator) */
};

/* Copy an internal array of level `level` into device memory dst_dev
 * (sizes as listed above).  For inspection and tests; synchronises. */
int mgfem_export(mgfem_handle h, int32_t what, int32_t level, double* dst_dev);

/* Grid size N_l of level `level` (0 = finest), or -1 if out of range. */
int32_t mgfem_level_n(mgfem_handle h, int32_t level);

/*
 * Apply `steps` smoothing steps of level `level` to x_dev for the right-hand
 * side b_dev (both device, (N_l+1)^2 float64; x is updated in place).
 * reverse != 0 applies the transposed step.  For tests of single sweeps.
 */
int mgfem_smooth(mgfem_handle h, int32_t level, double* x_dev, const double* b_dev,
                 int32_t steps, int32_t reverse);

/*
 * The Euclidean residual norms ||F - A u_m||_2, m = 0..cycles, of the last
 * mgfem_solve, mgfem_solve_mixed_bc or mgfem_adjoint on this handle, beside
 * the max-norm history those calls return (section 3.1 measures convergence
 * in the max norm; the l2 norm is reported with it).
 *  l2_hist_host : host, room for `capacity` float64 (may be NULL when
 *                 capacity is 0); receives the first min(capacity, count).
 *  count        : host, receives the number of entries of that history (may
 *                 be NULL).
 * Returns INVALID_ARG for a NULL handle or a negative capacity.
 */
int mgfem_residual_l2(mgfem_handle h, double* l2_hist_host, int32_t capacity, int32_t* count);

/*
 * The number of V-cycles each iteration of the last mgfem_solve,
 * mgfem_solve_mixed_bc or mgfem_adjoint on this handle ran, m = 1..cycles:
 * 1 for float64 iterations; for MGFEM_PRECISION_MIXED the float32 cycles of
 * each float64 step (params.inner_cycles, fewer where the residual history
 * shows that fewer reach the tolerance).
 *  cycles_host : host, room for `capacity` int32 (may be NULL when capacity
 *                is 0); receives the first min(capacity, count).
 *  count       : host, receives the number of iterations (may be NULL).
 * Returns INVALID_ARG for a NULL handle or a negative capacity.
 */
int mgfem_step_cycles(mgfem_handle h, int32_t* cycles_host, int32_t capacity, int32_t* count);

/* Per-level row counts: active rows, rows whose stencil is read from the
 * stored planes (the others are the interior Q1 stencil), extra-smoothing
 * vertices.  Any output pointer may be NULL. */
int mgfem_level_counts(mgfem_handle h, int32_t level, int64_t* n_active, int64_t* n_stored,
                       int64_t* n_cut);

/*
 * Kernel timing inside solves, for roofline measurements.  While enabled,
 * every launch of the profiled kernel class is bracketed by HIP events on the
 * handle's stream; after each solve the durations, the launch count and the
 * algorithmic bytes of those launches are accumulated.  Class 0 is the
 * float64 full-sweep kernel of the finest level, class 1 the float32 one of
 * the mixed-precision cycles; the algorithmic bytes per launch are, with w
 * the value size (8 or 4), 3w per active row (iterate read and written,
 * right-hand side) plus 9w per stored row, plus w per active coarse row when
 * the sweep applies the prolongation (the one flag byte per node it also
 * reads is not counted).
 *  enable : 0 off, 1 on, R in 2..1000: each timed launch is issued R times
 *           back to back between its two events (the sweep reads one iterate
 *           buffer and writes the other, so a repeat recomputes the same
 *           values) and its time is the elapsed time / R, which leaves out
 *           the dispatch gap an event pair adds to a single launch.
 * mgfem_profile resets the counters.
 */
int mgfem_profile(mgfem_handle h, int32_t enable);
int mgfem_profile_read(mgfem_handle h, int32_t kernel_class, int64_t* launches, double* total_ms,
                       double* alg_bytes);

/* Release the handle and all of its device memory. */
int mgfem_destroy(mgfem_handle h);

/* Static text for a status code. */
const char* mgfem_status_string(int code);

/* Text of the last error on h (thread-local last setup error when h is NULL). */
const char* mgfem_last_error(mgfem_handle h);

/*
 * Batched form: `count` independent problems (different psi and N) solved
 * together, float32 cycles inside float64 defect correction, with
 * per-problem convergence.  Setup builds every hierarchy and times two ways
 * of running the batch, keeping the faster (the autotuner): the tiled path,
 * where each step of the cycle is one launch over the tiles (cut groups,
 * coarse-map rows, ...) of every problem still iterating, with the kernels
 * and results of the single-problem mixed solve; or one persistent launch
 * whose workgroups take whole problems from a queue, with one of four
 * footprint widths.  Parameters are shared by all problems (both paths run
 * params.inner_cycles float32 cycles per float64 step, as mgfem_solve in
 * mixed precision; with rel_tol > 0 the tiled path runs a step with fewer
 * when no problem still iterating needs more by mgfem_solve's rule, and
 * MGFEM_FIXED_INNER=1 keeps the full count); the whole boundary is
 * Dirichlet.  MGFEM_BATCH_PATH=tiled or =persistent at set-up fixes the
 * choice.
 *  psi_dev[i] : device (N[i]+1)^2 float64.  N[i] as in mgfem_setup.
 */
int mgfem_setup_batched(int32_t count, const double* const* psi_dev, const int32_t* N,
                        const mgfem_params* p, void* stream, mgfem_handle* out);

/*
 *  f_dev[i], g_dev[i], u_dev[i] : device (N[i]+1)^2 float64.
 *  res_hist_host : host count*(max_cycles+1) float64 or NULL (row i for problem i).
 *  n_cycles      : host count int32 or NULL.
 * Returns OK when every problem converged, NOT_CONVERGED otherwise.
 */
int mgfem_solve_batched(mgfem_handle h, const double* const* f_dev, const double* const* g_dev,
                        double rel_tol, int32_t max_cycles, double* const* u_dev,
                        double* res_hist_host, int32_t* n_cycles);

/* The batched autotuner's choice: 0 for the tiled path, else the footprint
 * width (nodes per row of a workgroup's 1024-thread footprint on a colour
 * sub-lattice) of the persistent kernel; -1 for a handle that is not batched. */
int mgfem_batched_tile(mgfem_handle h);

#ifdef __cplusplus
}
#endif

#endif /* MGFEM_H */
