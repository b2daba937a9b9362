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
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/mgfem.h"

namespace mgfem {

constexpr int kFlagActive = 1;
constexpr int kFlagStored = 2;
constexpr int kFlagCut = 4;
// level-0 operator of a context: the assembled ghost-FEM matrix A, or the cut
// stiffness S of the global eigenproblem (section 5.2), whose stored rows get
// their diagonal scaled by 1 + kStiffnessShift so that the coarsest Cholesky
// factor exists (S alone vanishes on the constants)
constexpr int kOpAssembled = 0, kOpStiffness = 1;
constexpr double kStiffnessShift = 1e-12;

// cell type codes
constexpr int kExternal = 0, kTriangle = 1, kQuad = 2, kPentagon = 3, kInternal = 4,
              kSaddleSplit = 5, kSaddleHex = 6;

// Groups of cut vertices for the extra-smoothing kernel: each group owns the
// cut vertices of one spatial tile and carries the closure it needs (every cut
// vertex within 4 eta nodes of the tile), so that all 4 eta colour phases of
// one smoothing step run inside one workgroup's LDS.
struct CutPlan {
  bool ok = false;
  int ngroups = 0;
  int* g_info = nullptr;    // 9 ints per group: cl_off, cl_cnt, ext_off, ext_cnt, colour offsets[5]
  int* cl_node = nullptr;   // closure node index
  int* cl_q = nullptr;      // closure node position in the level's cut list
  uint8_t* cl_own = nullptr;
  int16_t* cl_nbr = nullptr;  // 8 per closure node: <cl_cnt closure slot, >= cl_cnt external slot, -1 none
  int* ext_src = nullptr;   // >= 0 node read from x; < 0 -(1+q) read from the cut-value snapshot
  double* cl_coef = nullptr;  // 9 per closure node: 8 off-diagonals, 1/diagonal
  float* cl_coef32 = nullptr;
  int max_cl = 0, max_ext = 0;
  int lds64 = 0, lds32 = 0;   // dynamic LDS of the largest group
};

// LDS layout of one cut group: values (closure, external, one zero slot),
// right-hand sides, inverse diagonals, 8 off-diagonal coefficients per node,
// 8 neighbour slots (int16) per node, and 64 bytes per lane of a wave where
// lanes with no node store what they loaded (so that the staging stores
// need no branch: 8 words of one lane lie 64 words apart); every block
// 16-byte aligned.
struct CutLds {
  int vals, b, invd, coef, refs, dump, total;
};
__host__ __device__ inline CutLds cut_lds_layout(int cl, int ext, int ts) {
  auto a16 = [](int v) { return (v + 15) & ~15; };
  CutLds L;
  L.vals = 0;
  L.b = L.vals + a16((cl + ext + 1) * ts);
  L.invd = L.b + a16(cl * ts);
  L.coef = L.invd + a16(cl * ts);
  L.refs = L.coef + a16(8 * cl * ts);
  L.dump = L.refs + 16 * cl;
  L.total = L.dump + 64 * 64;
  return L;
}

struct Level {
  int N = 0;
  int stride = 0;  // N + 1
  int64_t n = 0;   // (N+1)^2
  double* A = nullptr;
  float* A32 = nullptr;
  uint8_t* flags = nullptr;
  uint8_t* cellcut = nullptr;  // N*N, 1 on cut cells of this level
  double* X[2] = {nullptr, nullptr};  // ping-pong iterates (level 0: X[0] is the caller's)
  float* X32[2] = {nullptr, nullptr};
  double* b = nullptr;
  float* b32 = nullptr;
  int cur = 0;                // which X holds the current iterate (host-side state)
  int* cut_list = nullptr;    // concatenated colour lists of the cut vertices
  int cut_off[5] = {0, 0, 0, 0, 0};
  int* cutpos = nullptr;      // per node: position in cut_list, or -1
  double* snap = nullptr;     // cut-vertex values after the last full sweep
  float* snap32 = nullptr;
  CutPlan cp;
  int bbox[4] = {1, 0, 1, 0};  // i_lo, i_hi, j_lo, j_hi of active nodes (inclusive)
  int64_t n_active = 0, n_stored = 0;  // active rows, rows read from the planes
  int* tiles = nullptr;  // sweep tiles that hold an active node
  int ntiles = 0;
  int tile_shape = -1;
  // per sweep tile (in list order): the stored rows of its staged region
  // (region index, the 9 coefficients) and the cut vertices of its core
  // (region index, snapshot slot), so that a sweep reads no row and no
  // snapshot position from global memory between its colour phases
  int* tp_off = nullptr;  // ntiles + 1
  int* tp_idx = nullptr;
  double* tp_coef = nullptr;
  float* tp_coef32 = nullptr;
  int* tc_off = nullptr;  // ntiles + 1
  // per list entry: tile, first stored row, stored rows, first cut vertex, cut
  // vertices (and 3 unused): one 32-byte scalar load gives a sweep tile all of it
  int* tmeta = nullptr;
  // residual-restriction tiles of this level (coarse tiles of the next level
  // that hold an active coarse node)
  int* rr_tiles = nullptr;
  int rr_ntiles = 0;
  int* tc_idx = nullptr;
  int* tc_pos = nullptr;
  int tp_max = 0, tc_max = 0;
  bool empty() const { return bbox[0] > bbox[1]; }
};

// HIP-event timing of one kernel class inside a solve (see mgfem_profile)
struct Profiler {
  bool on = false;
  int repeat = 1;              // back-to-back launches between one event pair (time / repeat)
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<std::pair<int, double>> pending;  // (kernel class, algorithmic bytes)
  std::vector<hipEvent_t> cap_ev;  // pairs used by graph segments (created outside any capture)
  int64_t launches[4] = {0, 0, 0, 0};
  double ms[4] = {0, 0, 0, 0};
  double bytes[4] = {0, 0, 0, 0};
};

// One captured iteration of the solve loop (a cycle plus the reduction that
// yields the next residual norm), replayed with one graph launch.  The host
// bookkeeping (ping-pong parity of every level, reduction count) is a pure
// function of the state at capture, so a graph is keyed by that state and
// records the state it leaves behind.
struct ProfSlot {
  hipEvent_t beg, end;
  int kernel_class;
  double bytes;
};
// A timed launch is not captured: the entry keeps the launch itself and
// replays it between graph segments, bracketed by an event pair on the
// caller's stream (events around a graph launch cannot be timed).
struct GraphSeg {
  hipGraphExec_t exec = nullptr;
  std::function<void(hipStream_t)> launch;  // timed eager launch (exec null)
  int slot = -1;                            // index into GraphEntry::slots
};
struct GraphEntry {
  std::vector<GraphSeg> segs;
  std::vector<int> cur_after;  // loop state (ping-pong parities) after one replay
  int nred = 0;                // reductions per replay
  std::vector<ProfSlot> slots; // timed launches
  hipError_t err = hipSuccess; // first capture error
};

// Residual norms reach pinned host memory through a ring of records, one per
// reduction (slot = sequence number mod kRedSlots), so that a norm the host
// has not read yet survives the reductions of iterations queued after it.
constexpr int kRedSlots = 8;

// The coarse part of a cycle as a dense matrix (see k_coarse_apply): B maps
// the right-hand side of the first coarse level's active nodes to the iterate
// the coarse part leaves there, rows and columns in the order of idx.
constexpr int kMaxMapNodes = 4096;  // larger first coarse levels keep the single-workgroup cycle
struct CoarseMap {
  int level = -1;        // the level whose coarse part the map stands for (-1: no map)
  int n = 0;             // active nodes of that level
  int ld = 0;            // row stride (n rounded up to 16)
  int reps = 0;          // cycles of the coarse part the map stands for
  int* idx = nullptr;    // their grid indices on that level
  double* f64[2] = {nullptr, nullptr};  // forward and transposed cycles, float64
  float* f32 = nullptr;  // forward, float32 (the mixed-precision inner cycles)
};

// The coarsest levels run inside one workgroup, every array in LDS.
constexpr int kDesc = 32;  // ints per coarse-level descriptor
struct CoarsePlan {
  int lc = -1;            // first level of the single-workgroup part (-1: none)
  int* desc = nullptr;    // per level descriptor (see smoother.hip)
  double* coef = nullptr; // compact stored stencils of those levels
  float* coef32 = nullptr;
  int16_t* slot = nullptr;
  int16_t* cutl = nullptr;
  int16_t* actl = nullptr;  // active nodes per level and colour, as LDS-box indices
  double* inv = nullptr;  // inverse of the coarsest active block (float64)
  // the LDS content of the coarse part as a prebuilt image (zero vectors, the
  // lists, slots and rows, the coarsest inverse), float64 and float32 layouts
  unsigned char* img64 = nullptr;
  unsigned char* img32 = nullptr;
  int static64 = 0, static32 = 0;  // bytes of the static block (the image), whole 1 KB chunks
  int ndesc = 0;
  int lds64 = 0, lds32 = 0;
  CoarseMap map;
};

struct Stats {
  unsigned long long counts[7];
  unsigned long long snapped;
  unsigned long long active;
  unsigned long long min_theta_bits;   // float64 bits of the minimum (positive) theta
  unsigned long long max_lambda_bits;  // float64 bits of the maximum lambda
  int coarse_status;                   // 0 ok, 1 singular
  int coarse_n;
  unsigned long long dirichlet_cells;  // cut cells with a Dirichlet segment
};

// Batched solves on the tiled kernels ("team" path, team.hip): every launch
// covers the same step of the cycle for all problems of the batch, its
// workgroups taking (problem, unit) items of a work list.  Level-0 entry of
// one problem (plain device pointers; the data pointers change per solve).
struct TeamL0 {
  const double* A;
  const uint8_t* fl;
  int N, s;
  int64_t n;
  const double* M;
  const double* G;
  double h36;                // h^2 / 36, the interior mass stencil's scale
  const int* cut_list;
  int ncut;
  const double* cut_rows;    // 18 per cut-cell vertex: M row, G row
  double* F;                 // the load vector (level-0 right-hand side)
  double* U[2];              // float64 iterate buffers
  float* E[2];               // level-0 float iterates of the inner cycles
  float* r32;                // float residual: the inner cycle's right-hand side
  int i0, j0, ni, nj, gx;    // box of active nodes; 256 x 4 blocks per box row
  int nb;                    // blocks of the box (gx times the rows of blocks)
  double* part;              // one (max, sum) pair per box block
  const double* f;           // this solve's data and output
  const double* g;
  double* u_out;
  int ucur;                  // buffer of U that holds the final iterate (export)
};
constexpr int kTeamSweep = 0, kTeamCut = 1, kTeamRR = 2, kTeamMap = 3;  // float-cycle launch kinds
constexpr int kTeamCutRows = 0, kTeamRhs = 1, kTeamOuterFirst = 2, kTeamOuter = 3, kTeamExport = 4;
// float cycle (smoother.hip): entry size, one member's entry at level l,
// its work units there (-1: the member cannot take this path), one launch
size_t team_entry_bytes(int kind);
void team_entry(mgfem_ctx* m, int kind, int l, void* out);
int team_units(mgfem_ctx* m, int kind, int l);
int team_lds(mgfem_ctx* m, int kind, int l);  // dynamic LDS of its units
void team_launch(hipStream_t s, int kind, const void* tab, const int2* work, int nwork, int par, int parc,
                 int prolong, int lds);
// level 0 (cycle.hip): a member's entry (data pointers left null), the units
// of a level-0 launch kind, one launch, and the per-problem reduction of the
// box partials into out[2 p], out[2 p + 1] (max, sum of squares)
void team_l0_entry(mgfem_ctx* m, TeamL0* out);
int team_l0_units(const TeamL0& e, int kind);
void team_l0_launch(hipStream_t s, int kind, const TeamL0* tab, const int2* work, int nwork, int upar, int epar);
void team_reduce(hipStream_t s, const TeamL0* tab, const int* probs, int nprobs, double* out);
// the tiled path of a batched handle (team.hip): tables after the members'
// set-up, one solve (history count x (max_cycles + 1), cycles per problem,
// device time of the solve), release
int team_build(mgfem_ctx* b);
bool team_ok(const mgfem_ctx* b);
int team_solve(mgfem_ctx* b, const double* const* f, const double* const* g, double* const* u, double rel_tol,
               int max_cycles, std::vector<double>& hist, std::vector<int>& ncyc, float* ms);
void team_free(mgfem_ctx* b);

struct TeamPlan;  // team.hip

struct BatchDevice {
  void* probs = nullptr;  // per-problem layout records (built in smoother.hip)
  int* order = nullptr;   // problems by decreasing size (work-queue order)
  const double** f = nullptr;
  const double** g = nullptr;
  double** u = nullptr;
  double* hist = nullptr;
  int hist_cap = 0;
  int* ncyc = nullptr;
  unsigned int* queue = nullptr;
  int lds = 0;
  int tx = 0;  // autotuned footprint width (0: not tuned yet)
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
  double* cut_rows = nullptr;  // 18 per cut-cell vertex (M row, G row), in cut-list order
  double* GN = nullptr;        // 9 planes of the Neumann boundary mass (mixed boundaries only)
  double* cut_rows_n = nullptr;  // 9 per cut-cell vertex: the GN row, in cut-list order
  int op_kind = 0;               // kOpAssembled or kOpStiffness
  double* Kp = nullptr;          // kOpStiffness: 9 planes of K = int_{Gamma_D} (n.grad phi_i)(n.grad phi_j)
  double* cut_rows_k = nullptr;  // kOpStiffness: the K rows of the cut-cell vertices
  double lambda_global = 0.0;    // MGFEM_STAB_GLOBAL: gamma C
  double C_global = 0.0;         // MGFEM_STAB_GLOBAL: C
  double* F = nullptr;
  double* F64tmp = nullptr;  // outer residual / scratch on level 0
  double* zero = nullptr;    // all-zero vector of level 0
  double* lam = nullptr;     // adjoint state when the caller passes none
  // coarsest exact solve
  double* coarse_L = nullptr;  // cn x cn lower Cholesky factor, then its inverse
  int* coarse_idx = nullptr;   // cn node indices
  int coarse_n = 0;
  mgfem::CoarsePlan cplan;
  int tile_cfg = 0;            // sweep tile shape selection for large levels
  // reductions
  double* red_partial = nullptr;  // one (max, sum) pair per block of the level-0 box kernels
  double* red_out = nullptr;      // 2 doubles on device
  double* red_host = nullptr;     // pinned: kRedSlots records (max, sum of squares, sequence number, unused)
  double red_seq = 0.0;           // sequence number of the last reduction launched
  double* red_seq_dev = nullptr;  // the same count kept on the device (bumped by each reduction kernel)
  double* sweep_part = nullptr;   // per-tile partials of the fused residual norm
  unsigned int* sweep_counter = nullptr;
  mgfem::Stats* stats = nullptr;  // device
  mgfem_info info{};
  std::vector<void*> allocs;
  mgfem::Profiler prof;
  // graph replay of the solve loop
  bool use_graphs = true;
  bool graphs_failed = false;       // a capture failed: run this context eagerly
  hipStream_t cap_stream = nullptr; // stream the iterations are captured on
  mgfem::GraphEntry* capturing = nullptr;
  std::map<std::vector<int>, mgfem::GraphEntry> graphs;
  double* x0 = nullptr;             // level-0 iterate owned by the library (ping-pong partner of lv[0].X[1])
  int u_cur = 0;                    // mixed precision: which level-0 float64 buffer holds u
  double f_l2 = 0.0;                // ||F||_2 of the right-hand side the last solve assembled
  std::vector<double> l2_hist;      // ||F - A u_m||_2 of the last solve or adjoint, m = 0..cycles
  std::vector<int> step_cycles;     // V-cycles run by each iteration of the last solve or adjoint
  std::string last_error;
  int device = 0;                   // device that was current at set-up
  bool batched_member = false;
  std::vector<mgfem_ctx*> members;  // batched handle: one context per problem
  mgfem::BatchDevice batch;
  mgfem::TeamPlan* team = nullptr;  // batched handle: the tiled path's tables (null or !ok: not available)
};

namespace mgfem {


constexpr int kDotBlocks = 4096;  // blocks of the grid-stride dot product
// (max, sum) pairs of the reduction buffer: the 2D box kernels of level 0
// (256 x 4 nodes per block) or the dot product, whichever needs more
inline int64_t red_pairs(int N) {
  const int64_t box = (int64_t)((N + 256) / 256) * ((N + 4) / 4);
  return (box > kDotBlocks ? box : kDotBlocks) + 2;
}

void set_setup_error(const std::string& msg);  // text returned by mgfem_last_error(NULL)

// memory helpers (record the allocation on the context)
hipError_t ctx_alloc(mgfem_ctx* c, void** p, size_t bytes);
template <class T>
hipError_t ctx_alloc_t(mgfem_ctx* c, T** p, size_t count) {
  return ctx_alloc(c, reinterpret_cast<void**>(p), count * sizeof(T));
}

// setup stages (geometry.hip, hierarchy.hip)
int setup_geometry(mgfem_ctx* c, const double* psi_in, const double* chi_in);
int setup_hierarchy(mgfem_ctx* c, const double* psi_in, const double* chi_in);
// coarse level l assembled from scratch on its own grid from the fine input
// level set (injection, snapping, classification, stabilisation, assembly):
// fills lv[l].A, flags and cellcut (MGFEM_COARSE_REDISCRETISED)
int assemble_level(mgfem_ctx* c, int l, const double* psi_in, const double* chi_in);

// solve stages (cycle.hip)
// F = M f + G g, and its norm (max, sum of squares) as the next reduction
void launch_rhs(mgfem_ctx* c, const double* f, const double* g, const double* gN, double* F);
// mixed outer step: u_out = u + e, r = F - A u_out, r32 = float(r), z32 = 0 on
// the active nodes, and the norm of r as the next reduction (F = lv[0].b)
void launch_outer(mgfem_ctx* c, const double* u, const float* e, double* u_out, float* r32, float* z32);
// y = M x and y = G^T x on the fine grid (every node of y written)
void launch_mass_apply(mgfem_ctx* c, const double* x, double* y);
void launch_gt_apply(mgfem_ctx* c, const double* x, double* y);
int build_cut_rows(mgfem_ctx* c);  // gathered M, G (and GN) rows of the cut-cell vertices
void launch_gn_apply(mgfem_ctx* c, const double* x, double* y);  // y = GN x
void launch_k_apply(mgfem_ctx* c, const double* x, double* y);   // y = K x (kOpStiffness)
// vector kernels of the global eigenproblem's Lanczos iteration (stabilise.hip)
void launch_start_vector(mgfem_ctx* c, double* x);                  // seeded values on the active nodes
void launch_active_ones(mgfem_ctx* c, double* x);                   // 1 on the active nodes, 0 elsewhere
void launch_lanczos_update(mgfem_ctx* c, double* w, const double* q, const double* qp, double a, double b);
void launch_shift_active(mgfem_ctx* c, double* w, double v);         // w -= v on the active nodes
void launch_scale(mgfem_ctx* c, double* dst, const double* src, double s);
void launch_axpy(mgfem_ctx* c, double* y, const double* x, double a);
void launch_mask_inactive(mgfem_ctx* c, double* u);
void launch_residual_norm(mgfem_ctx* c, const double* F, const double* u, double* r_out);
void launch_dot_reduce(mgfem_ctx* c, const double* a, const double* b);
void launch_zero(mgfem_ctx* c, double* p, int64_t n);
void launch_copy(mgfem_ctx* c, double* dst, const double* src, int64_t n);
void launch_sub_active(mgfem_ctx* c, double* d, const double* a, const double* b);
void launch_u8_to_f64(mgfem_ctx* c, const uint8_t* s, double* d, int64_t n);
// level-0 bounding-box transfers: dst = src (or 0) on the box of active nodes;
// export writes every node of dst (the box from src, zero outside)
void launch_box_copy(mgfem_ctx* c, double* dst, const double* src);
void launch_export(mgfem_ctx* c, double* dst, const double* src);

struct CycleOpts {
  bool reverse = false;           // transposed cycle (adjoint)
  bool fp32 = false;              // float inner cycle
  bool first_sweep_done = false;  // the first level-0 sweep already ran (first_sweep_with_norm)
};
// first pre-smoothing sweep of level 0 (float64, forward) that also reduces the
// residual norm of its incoming iterate into red_out
void first_sweep_with_norm(mgfem_ctx* c);
// one cycle on level 0 from its current iterate X[cur] and right-hand side b
void run_cycle(mgfem_ctx* c, const CycleOpts& o);
void smooth_level(mgfem_ctx* c, int l, bool reverse, bool fp32);
void gather_snap(mgfem_ctx* c, int l, bool fp32);
int build_plans(mgfem_ctx* c);  // cut groups and the coarse single-workgroup layout
// the coarse part as a dense map (forward and, unless forward_only, transposed,
// float64; float32 forward for mixed precision); skipped for large first
// coarse levels and when MGFEM_NO_COARSE_MAP=1 at set-up
int build_coarse_map(mgfem_ctx* c, bool forward_only);
// the device-side address of the static scratch array of the current device,
// looked up once per device (noalloc.hip); *device receives that device
int scratch_init(int* device);
// mgfem_setup for one problem of a batched handle (forward coarse map only)
int setup_member(const double* psi_dev, int32_t N, const mgfem_params* p, void* stream, mgfem_handle* out);
int build_tile_lists(mgfem_ctx* c);
// sweep tile shapes, all with 512 threads (a workgroup's load phase is bound
// by the memory instructions each wave issues, so more waves per tile start
// the phases sooner): 64 x 32 on a finest level with N >= 2048, 64 x 16 on
// the other levels with N >= 1024, 16 x 16 below (measured on MI355X)
constexpr int kShapeFinest = 0, kShapeLarge = 1, kShapeSmall = 2;
inline int sweep_shape(const mgfem_ctx* c, int l) {
  const int N = c->lv[l].N;
  if (l == 0 && N >= 2048) return kShapeFinest;
  return N >= 1024 ? kShapeLarge : kShapeSmall;
}
void set_kernel_attributes();
// batched solves (layout and launch in smoother.hip)
void build_batch_layout(std::vector<mgfem_ctx*>& members, std::vector<unsigned char>& probs_bytes, int& lds);
float launch_batched(mgfem_ctx* b, BatchDevice& d, int count, double tol, int max_cycles, int tx);
// profiling: a launch timed with HIP events (inside a capture it stays an
// eager launch of the replay, see GraphSeg), and the collection of the timings
void prof_launch(mgfem_ctx* c, int kernel_class, double bytes, std::function<void(hipStream_t)> launch);
void prof_collect(mgfem_ctx* c);
void drop_graphs(mgfem_ctx* c);

}  // namespace mgfem

#define MGFEM_HIP_TRY(expr)                                                   \
  do {                                                                        \
    hipError_t _e = (expr);                                                   \
    if (_e != hipSuccess) {                                                   \
      c->last_error = std::string(#expr) + ": " + hipGetErrorString(_e);      \
      return _e == hipErrorOutOfMemory ? MGFEM_ERR_OOM : MGFEM_ERR_HIP;       \
    }                                                                         \
  } while (0)
