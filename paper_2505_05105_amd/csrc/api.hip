// C ABI of the library: argument checks, the hierarchy's allocation, the
// solve / adjoint drivers and their convergence bookkeeping.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <new>

#include "mgfem_internal.h"

using namespace mgfem;

namespace {

thread_local std::string g_setup_error;

int fail(mgfem_ctx* c, int code, const std::string& msg) {
  if (c) c->last_error = msg;
  else g_setup_error = msg;
  return code;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int check_params(const mgfem_params& p, int N, std::string& why) {
  if (p.stab_rule < 0 || p.stab_rule > 3) return why = "stab_rule", 1;
  if (p.stab_rule == MGFEM_STAB_GLOBAL && p.coarse_op == MGFEM_COARSE_REDISCRETISED)
    return why = "the global stabilisation rule needs Galerkin coarse operators", 1;
  if (p.stab_rule != MGFEM_STAB_FIXED && !(p.gamma > 1.0))
    return why = "gamma must exceed 1 (coercivity, section 4.4)", 1;
  if (p.stab_rule == MGFEM_STAB_FIXED && !(p.lambda_fixed > 0.0)) return why = "lambda_fixed", 1;
  if (!(p.snap_alpha > 0.0)) return why = "snap_alpha", 1;
  if (p.nu1 < 0 || p.nu2 < 0 || p.nu1 + p.nu2 == 0 || p.eta < 0 || p.nu1 > 64 || p.nu2 > 64 || p.eta > 64)
    return why = "nu1/nu2/eta", 1;
  if (p.coarsest_n < 1 || p.coarsest_n > 16) return why = "coarsest_n must be in [1, 16]", 1;
  if (p.precision != MGFEM_PREC_FP64 && p.precision != MGFEM_PREC_MIXED) return why = "precision", 1;
  if (p.precision == MGFEM_PREC_MIXED && (p.inner_cycles < 1 || p.inner_cycles > 16))
    return why = "inner_cycles must be 1..16", 1;
  if (p.cycle != MGFEM_CYCLE_V && p.cycle != MGFEM_CYCLE_W && p.cycle != MGFEM_CYCLE_TWO_GRID)
    return why = "cycle", 1;
  if (p.cycle == MGFEM_CYCLE_TWO_GRID && (p.coarse_cycles < 1 || p.coarse_cycles > 1000))
    return why = "coarse_cycles must be 1..1000", 1;
  if (p.coarse_op != MGFEM_COARSE_GALERKIN && p.coarse_op != MGFEM_COARSE_REDISCRETISED) return why = "coarse_op", 1;
  const double wx = p.x_hi - p.x_lo, wy = p.y_hi - p.y_lo;
  if (!(wx > 0.0) || !(wy > 0.0) || std::fabs(wx - wy) > 1e-12 * wx)
    return why = "the box must be a non-empty square", 1;
  if (N < 2 * p.coarsest_n || N % p.coarsest_n || !is_pow2(N / p.coarsest_n) || N > (1 << 15))
    return why = "N must be coarsest_n times a power of two (>= 2), at most 32768", 1;
  return 0;
}

}  // namespace

namespace mgfem {
void set_setup_error(const std::string& msg) { g_setup_error = msg; }

hipError_t ctx_alloc(mgfem_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return e;
  c->allocs.push_back(*p);
  return hipMemsetAsync(*p, 0, bytes, c->s);
}
}  // namespace mgfem

namespace mgfem {
// capture segments: close the running capture into a graph segment
static void cap_fail(mgfem_ctx* c, hipError_t e, const char* what) {
  GraphEntry& g = *c->capturing;
  if (e != hipSuccess && g.err == hipSuccess) {
    g.err = e;
    c->last_error = std::string("graph capture: ") + what + ": " + hipGetErrorString(e);
  }
}
static void seg_close(mgfem_ctx* c, int slot) {
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
  cap_fail(c, e, "hipStreamEndCapture");
  if (e == hipSuccess && graph) {
    size_t nodes = 0;
    e = hipGraphGetNodes(graph, nullptr, &nodes);
    cap_fail(c, e, "hipGraphGetNodes");
    if (e == hipSuccess && nodes > 0) {
      GraphSeg sg;
      sg.slot = slot;
      e = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
      cap_fail(c, e, "hipGraphInstantiate");
      if (e == hipSuccess) c->capturing->segs.push_back(sg);
    }
  }
  if (graph) (void)hipGraphDestroy(graph);
}
static void seg_open(mgfem_ctx* c) {
  cap_fail(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
}

void prof_launch(mgfem_ctx* c, int kernel_class, double bytes, std::function<void(hipStream_t)> launch) {
  Profiler& P = c->prof;
  if (c->capturing) {
    GraphEntry& g = *c->capturing;
    const size_t i = g.slots.size();
    if (2 * (i + 1) > P.cap_ev.size()) {
      cap_fail(c, hipErrorInvalidValue, "too many timed launches in one iteration");
      return;
    }
    g.slots.push_back(ProfSlot{P.cap_ev[2 * i], P.cap_ev[2 * i + 1], kernel_class, bytes});
    seg_close(c, -1);
    GraphSeg sg;
    sg.launch = std::move(launch);
    sg.slot = (int)i;
    g.segs.push_back(std::move(sg));
    seg_open(c);
    return;
  }
  const int slot = (int)P.pending.size();
  while ((int)P.ev.size() < 2 * (slot + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      launch(c->s);
      return;
    }
    P.ev.push_back(e);
  }
  (void)hipEventRecord(P.ev[2 * slot], c->s);
  for (int r = 0; r < P.repeat; ++r) launch(c->s);
  (void)hipEventRecord(P.ev[2 * slot + 1], c->s);
  P.pending.push_back({kernel_class, bytes});
}
void prof_collect(mgfem_ctx* c) {
  Profiler& P = c->prof;
  if (P.pending.empty()) return;
  (void)hipStreamSynchronize(c->s);
  for (size_t i = 0; i < P.pending.size(); ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, P.ev[2 * i], P.ev[2 * i + 1]) != hipSuccess) continue;
    const int k = P.pending[i].first;
    P.launches[k] += 1;
    P.ms[k] += ms / P.repeat;
    P.bytes[k] += P.pending[i].second;
  }
  P.pending.clear();
}
// timings of the launches inside one finished graph replay
static int prof_collect_graph(mgfem_ctx* c, const GraphEntry& g) {
  if (g.slots.empty()) return MGFEM_OK;
  Profiler& P = c->prof;
  MGFEM_HIP_TRY(hipEventSynchronize(g.slots.back().end));
  for (const ProfSlot& sl : g.slots) {
    float ms = 0.f;
    MGFEM_HIP_TRY(hipEventElapsedTime(&ms, sl.beg, sl.end));
    P.launches[sl.kernel_class] += 1;
    P.ms[sl.kernel_class] += ms / P.repeat;
    P.bytes[sl.kernel_class] += sl.bytes;
  }
  return MGFEM_OK;
}
static void destroy_graph(GraphEntry& g) {
  for (GraphSeg& sg : g.segs)
    if (sg.exec) (void)hipGraphExecDestroy(sg.exec);
  g.segs.clear();
  g.slots.clear();  // the events belong to the profiler
}
void drop_graphs(mgfem_ctx* c) {
  for (auto& kv : c->graphs) destroy_graph(kv.second);
  c->graphs.clear();
}
}  // namespace mgfem

static void free_ctx(mgfem_ctx* c) {
  if (!c) return;
  if (c->s) (void)hipStreamSynchronize(c->s);
  else (void)hipDeviceSynchronize();
  for (hipEvent_t e : c->prof.ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->prof.cap_ev) (void)hipEventDestroy(e);
  mgfem::drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (void* q : c->allocs) (void)hipFree(q);
  if (c->red_host) (void)hipHostFree(c->red_host);
  delete c;
}

extern "C" {

int mgfem_default_params(mgfem_params* p) {
  if (!p) return MGFEM_ERR_INVALID_ARG;
  std::memset(p, 0, sizeof(*p));
  p->stab_rule = MGFEM_STAB_PAPER;
  p->gamma = 2.0;
  p->lambda_fixed = 0.0;
  p->snap_alpha = 1.75;
  p->nu1 = 2;
  p->nu2 = 1;
  p->eta = 4;
  p->coarsest_n = 4;
  p->precision = MGFEM_PREC_FP64;
  p->cycle = MGFEM_CYCLE_V;
  p->coarse_cycles = 40;
  p->coarse_op = MGFEM_COARSE_GALERKIN;
  p->inner_cycles = 3;
  p->x_lo = -1.0;
  p->y_lo = -1.0;
  p->x_hi = 1.0;
  p->y_hi = 1.0;
  return MGFEM_OK;
}

const char* mgfem_status_string(int code) {
  switch (code) {
    case MGFEM_OK: return "ok";
    case MGFEM_ERR_INVALID_ARG: return "invalid argument";
    case MGFEM_ERR_OOM: return "out of device memory";
    case MGFEM_ERR_HIP: return "HIP runtime error";
    case MGFEM_ERR_NOT_CONVERGED: return "not converged within max_cycles";
    case MGFEM_ERR_DIVERGED: return "diverged";
    case MGFEM_ERR_SINGULAR_COARSE: return "coarsest matrix not positive definite";
    case MGFEM_ERR_EMPTY_DOMAIN: return "empty domain";
    case MGFEM_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

const char* mgfem_last_error(mgfem_handle h) {
  return h ? h->last_error.c_str() : g_setup_error.c_str();
}

}  // extern "C"

namespace {

int global_constant(const double* psi, const double* chi, int32_t N, const mgfem_params& p, void* stream,
                    double* C_out, int* iters_out);

int setup_impl(const double* psi_dev, const double* chi_dev, int32_t N, const mgfem_params* pin, void* stream,
               mgfem_handle* out, int op_kind = kOpAssembled, bool member = false) {
  if (!out) return fail(nullptr, MGFEM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!psi_dev) return fail(nullptr, MGFEM_ERR_INVALID_ARG, "psi_dev is NULL");
  mgfem_params p;
  if (pin) p = *pin;
  else mgfem_default_params(&p);
  std::string why;
  if (check_params(p, N, why)) return fail(nullptr, MGFEM_ERR_INVALID_ARG, "invalid parameter: " + why);
  double C_global = 0.0;
  int global_iters = 0;
  if (p.stab_rule == MGFEM_STAB_GLOBAL && op_kind == kOpAssembled) {
    const int rc = global_constant(psi_dev, chi_dev, N, p, stream, &C_global, &global_iters);
    if (rc != MGFEM_OK) return rc;  // the message is already set
  }
  mgfem_ctx* c = new (std::nothrow) mgfem_ctx();
  if (!c) return fail(nullptr, MGFEM_ERR_OOM, "host allocation failed");
  c->p = p;
  c->op_kind = op_kind;
  c->C_global = C_global;
  c->lambda_global = p.gamma * C_global;
  c->s = reinterpret_cast<hipStream_t>(stream);
  c->N = N;
  c->h = (p.x_hi - p.x_lo) / N;
  for (int n = N; n >= p.coarsest_n; n /= 2) {
    Level L;
    L.N = n;
    L.stride = n + 1;
    L.n = (int64_t)(n + 1) * (n + 1);
    c->lv.push_back(L);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = MGFEM_OK;
  auto bail = [&](int code) {
    std::string msg = c->last_error;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    free_ctx(c);
    return fail(nullptr, code, msg);
  };
#define SETUP_TRY(x)                                               \
  do {                                                             \
    hipError_t _e = (x);                                           \
    if (_e != hipSuccess) {                                        \
      c->last_error = std::string(#x) + ": " + hipGetErrorString(_e); \
      return bail(_e == hipErrorOutOfMemory ? MGFEM_ERR_OOM : MGFEM_ERR_HIP); \
    }                                                              \
  } while (0)
  SETUP_TRY(hipEventCreate(&e0));
  SETUP_TRY(hipEventCreate(&e1));
  SETUP_TRY(hipEventRecord(e0, c->s));
  SETUP_TRY(ctx_alloc_t(c, &c->stats, 1));
  {
    Stats init{};
    init.min_theta_bits = 0x7ff0000000000000ull;
    SETUP_TRY(hipMemcpyAsync(c->stats, &init, sizeof(init), hipMemcpyHostToDevice, c->s));
  }
  const int64_t n0 = c->lv[0].n;
  SETUP_TRY(ctx_alloc_t(c, &c->F, n0));
  SETUP_TRY(ctx_alloc_t(c, &c->F64tmp, n0));
  SETUP_TRY(ctx_alloc_t(c, &c->zero, n0));
  SETUP_TRY(ctx_alloc_t(c, &c->lam, n0));
  // one (max, sum) pair per block of the level-0 box kernels (256 x 4 nodes)
  SETUP_TRY(ctx_alloc_t(c, &c->red_partial, 2 * red_pairs(N)));
  SETUP_TRY(ctx_alloc_t(c, &c->red_out, 2));
  SETUP_TRY(ctx_alloc_t(c, &c->red_seq_dev, 1));
  SETUP_TRY(ctx_alloc_t(c, &c->sweep_counter, 1));
  {
    // one partial pair per level-0 sweep tile (every tile shape holds at least 16 x 16 nodes)
    const int64_t tiles = (int64_t)(N / 16 + 2) * (N / 16 + 2);
    SETUP_TRY(ctx_alloc_t(c, &c->sweep_part, 2 * tiles));
  }
  // the ring of norm records, and one more record for mgfem_misfit_noalloc
  SETUP_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->red_host), 4 * (kRedSlots + 1) * sizeof(double)));
  for (int q = 0; q < 4 * (kRedSlots + 1); ++q) c->red_host[q] = 0.0;
  if (scratch_init(&c->device) != MGFEM_OK) {
    c->last_error = "hipGetDevice failed";
    return bail(MGFEM_ERR_HIP);
  }
  {
    const char* env = std::getenv("MGFEM_NO_GRAPHS");
    c->use_graphs = !(env && env[0] && env[0] != '0');
  }
  rc = setup_geometry(c, psi_dev, chi_dev);
  if (rc != MGFEM_OK) return bail(rc);
  rc = setup_hierarchy(c, psi_dev, chi_dev);
  if (rc != MGFEM_OK) return bail(rc);
  SETUP_TRY(hipEventRecord(e1, c->s));
  Stats st{};
  SETUP_TRY(hipMemcpyAsync(&st, c->stats, sizeof(st), hipMemcpyDeviceToHost, c->s));
  SETUP_TRY(hipStreamSynchronize(c->s));
  float ms = 0.f;
  SETUP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  e0 = e1 = nullptr;
  if (chi_dev && op_kind == kOpAssembled && st.dirichlet_cells == 0) {
    c->last_error = "no interface segment is a Dirichlet segment: with Neumann data on the whole boundary the "
                    "problem is singular";
    return bail(MGFEM_ERR_INVALID_ARG);
  }
  if (st.coarse_status != 0) {
    c->last_error = "non-positive pivot in the Cholesky factor of the coarsest operator";
    return bail(MGFEM_ERR_SINGULAR_COARSE);
  }
  if (st.coarse_n > 512) {
    c->last_error = "coarsest grid has more than 512 active nodes";
    return bail(MGFEM_ERR_INVALID_ARG);
  }
  c->coarse_n = st.coarse_n;
  rc = build_plans(c);
  if (rc != MGFEM_OK) return bail(rc);
  rc = build_cut_rows(c);
  if (rc != MGFEM_OK) return bail(rc);
  rc = build_coarse_map(c, member);  // batch members run forward float cycles only
  if (rc != MGFEM_OK) return bail(rc);
  SETUP_TRY(hipStreamSynchronize(c->s));
  mgfem_info& I = c->info;
  I.N = N;
  I.n_levels = (int)c->lv.size();
  I.n_active = (int64_t)st.active;
  for (int t = 0; t < 7; ++t) I.n_cells_by_type[t] = (int64_t)st.counts[t];
  I.n_snapped = (int64_t)st.snapped;
  I.n_cut_vertices = c->lv[0].cut_off[4];
  I.coarse_n = st.coarse_n;
  double mt, ml;
  std::memcpy(&mt, &st.min_theta_bits, 8);
  std::memcpy(&ml, &st.max_lambda_bits, 8);
  I.min_theta = std::isinf(mt) ? 0.0 : mt;
  I.max_lambda = ml;
  I.setup_ms = ms;
  I.global_C = C_global;
  I.global_iters = global_iters;
#undef SETUP_TRY
  *out = c;
  return MGFEM_OK;
}

}  // namespace

namespace mgfem {
int setup_member(const double* psi_dev, int32_t N, const mgfem_params* p, void* stream, mgfem_handle* out) {
  return setup_impl(psi_dev, nullptr, N, p, stream, out, kOpAssembled, true);
}
}  // namespace mgfem

extern "C" {

int mgfem_setup(const double* psi_dev, int32_t N, const mgfem_params* p, void* stream, mgfem_handle* out) {
  return setup_impl(psi_dev, nullptr, N, p, stream, out);
}

int mgfem_setup_mixed_bc(const double* psi_dev, const double* chi_dev, int32_t N, const mgfem_params* p,
                         void* stream, mgfem_handle* out) {
  return setup_impl(psi_dev, chi_dev, N, p, stream, out);
}

int mgfem_query(mgfem_handle h, mgfem_info* info) {
  if (!h || !info) return MGFEM_ERR_INVALID_ARG;
  *info = h->info;
  return MGFEM_OK;
}

int32_t mgfem_level_n(mgfem_handle h, int32_t level) {
  if (!h || level < 0 || level >= (int)h->lv.size()) return -1;
  return h->lv[level].N;
}

int mgfem_destroy(mgfem_handle h) {
  if (!h) return MGFEM_ERR_INVALID_ARG;
  for (mgfem_ctx* m : h->members) free_ctx(m);
  h->members.clear();
  team_free(h);
  free_ctx(h);
  return MGFEM_OK;
}

}  // extern "C"

namespace {

// read the (max, sum of squares) of reduction number `want` (default: the
// last one launched) to the host
int read_norm(mgfem_ctx* c, double& mx, double& l2, double* raw_sum = nullptr, double want = -1.0) {
  // the reduction kernel writes (max, sum of squares, sequence number) into
  // its record of pinned host memory; wait for this reduction's number, then
  // fall back to a stream synchronisation if it does not arrive (a failed
  // launch)
  if (want < 0.0) want = c->red_seq;
  volatile double* h = c->red_host + 4 * (int)((long long)want % kRedSlots);
  const auto t0 = std::chrono::steady_clock::now();
  while (h[2] != want) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(200)) {
      MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
      MGFEM_HIP_TRY(hipGetLastError());
      if (h[2] != want) {
        c->last_error = "residual norm " + std::to_string(want) + " did not arrive (last " +
                        std::to_string(h[2]) + ")";
        return MGFEM_ERR_HIP;
      }
      break;
    }
  }
  mx = h[0];
  l2 = std::sqrt(h[1]);
  if (raw_sum) *raw_sum = h[1];
  return MGFEM_OK;
}

// cycles on A x = b (x, b on level 0) until the relative tolerance is met;
// x is the caller's buffer and receives the result
// Enqueue one iteration of the solve loop: a cycle from the current iterate
// and the reduction that gives the residual norm of the next one.
//  float64 forward: the rest of the cycle (its first sweep ran in the previous
//    iteration), then the first sweep of the next cycle with the fused norm of
//    its incoming iterate (speculative: discarded when the loop stops);
//  mixed: inner_cycles float cycles on the float residual of the previous
//    step (the first from zero), then one fused pass u += e, r = F - A u
//    (float64), its float copy, the next zero start iterate and the norm;
//  adjoint: a transposed cycle, then the residual norm.
struct IterKind {
  bool mixed, reverse, first_done;
  int inner;  // mixed: float32 cycles of this step
};
void enqueue_iteration(mgfem_ctx* c, const IterKind& k) {
  Level& L0 = c->lv[0];
  if (k.mixed) {
    // the inner right-hand side b32 and the zero start iterate X32[cur] were
    // written by the previous outer step
    CycleOpts o;
    o.fp32 = true;
    o.reverse = k.reverse;
    for (int q = 0; q < k.inner; ++q) run_cycle(c, o);
    const int ce = L0.cur;
    launch_outer(c, L0.X[c->u_cur], L0.X32[ce], L0.X[1 - c->u_cur], L0.b32, L0.X32[1 - ce]);
    c->u_cur = 1 - c->u_cur;
    L0.cur = 1 - ce;
  } else if (k.reverse) {
    CycleOpts o;
    o.reverse = true;
    run_cycle(c, o);
    launch_residual_norm(c, L0.b, L0.X[L0.cur], nullptr);
  } else {
    CycleOpts o;
    o.first_sweep_done = k.first_done;
    run_cycle(c, o);
    first_sweep_with_norm(c);
  }
}

// host-side state that an iteration reads and advances: the ping-pong parity
// of every level and of the float64 level-0 iterate of the mixed solve
std::vector<int> loop_state(const mgfem_ctx* c) {
  std::vector<int> st;
  for (const Level& L : c->lv) st.push_back(L.cur);
  st.push_back(c->u_cur);
  return st;
}
void set_loop_state(mgfem_ctx* c, const std::vector<int>& st) {
  for (size_t l = 0; l < c->lv.size(); ++l) c->lv[l].cur = st[l];
  c->u_cur = st[c->lv.size()];
}

std::vector<int> graph_key(mgfem_ctx* c, const IterKind& k) {
  std::vector<int> key{k.mixed, k.reverse, k.first_done, c->prof.on ? 1 : 0, k.inner};
  for (int v : loop_state(c)) key.push_back(v);
  return key;
}

// Run one iteration: replay its graph (captured on first use) or launch it
// eagerly.  Returns the graph used, or null.
int run_iteration(mgfem_ctx* c, const IterKind& k, const GraphEntry** used) {
  *used = nullptr;
  if (!c->use_graphs || c->graphs_failed) {
    enqueue_iteration(c, k);
    MGFEM_HIP_TRY(hipGetLastError());
    return MGFEM_OK;
  }
  const std::vector<int> key = graph_key(c, k);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    if (!c->cap_stream) MGFEM_HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    // the capture stream starts after the work already queued on the caller's
    // stream only through the graph launch below, which is stream-ordered
    if (c->prof.on && c->prof.cap_ev.empty()) {
      // timed launches per iteration: three finest sweeps (W-cycle: the same)
      for (int q = 0; q < 8; ++q) {
        hipEvent_t e;
        MGFEM_HIP_TRY(hipEventCreate(&e));
        c->prof.cap_ev.push_back(e);
      }
    }
    GraphEntry g;
    hipStream_t user = c->s;
    const double seq0 = c->red_seq;
    const std::vector<int> st0 = loop_state(c);
    c->s = c->cap_stream;
    c->capturing = &g;
    seg_open(c);
    if (g.err == hipSuccess) {
      enqueue_iteration(c, k);
      seg_close(c, -1);
    }
    c->capturing = nullptr;
    c->s = user;
    g.nred = (int)(c->red_seq - seq0 + 0.5);
    g.cur_after = loop_state(c);
    c->red_seq = seq0;
    set_loop_state(c, st0);
    (void)hipGetLastError();
    if (g.err != hipSuccess) {
      // capture is not available here: run this context eagerly from now on
      // (the reason stays readable through mgfem_last_error)
      hipStreamCaptureStatus st;
      if (hipStreamIsCapturing(c->cap_stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(c->cap_stream, &junk);
        if (junk) (void)hipGraphDestroy(junk);
      }
      (void)hipGetLastError();
      destroy_graph(g);
      c->graphs_failed = true;
      std::fprintf(stderr, "mgfem: %s; iterations run without graphs\n", c->last_error.c_str());
      enqueue_iteration(c, k);
      MGFEM_HIP_TRY(hipGetLastError());
      return MGFEM_OK;
    }
    it = c->graphs.emplace(key, std::move(g)).first;
  }
  GraphEntry& g = it->second;
  MGFEM_HIP_TRY(hipGetLastError());
  for (const GraphSeg& sg : g.segs) {
    if (sg.launch) {
      MGFEM_HIP_TRY(hipEventRecord(g.slots[sg.slot].beg, c->s));
      for (int r = 0; r < c->prof.repeat; ++r) sg.launch(c->s);
      MGFEM_HIP_TRY(hipEventRecord(g.slots[sg.slot].end, c->s));
    } else {
      MGFEM_HIP_TRY(hipGraphLaunch(sg.exec, c->s));
    }
  }
  c->red_seq += g.nred;
  set_loop_state(c, g.cur_after);
  *used = &g;
  return MGFEM_OK;
}

// x: caller's iterate (input when warm, output), b: level-0 right-hand side
// (device buffer owned by the context).  The loop runs on the library's own
// level-0 buffers so that captured graphs never see a caller pointer.
int iterate(mgfem_ctx* c, double* x, const double* b, double rel_tol, int max_cycles, bool reverse,
            bool mixed, bool warm, double bnorm, double* hist, int* ncyc) {
  Level& L0 = c->lv[0];
  // the loop reads its own history (step lengths, queueing), so it keeps one
  // when the caller asks for none
  std::vector<double> own_hist;
  if (!hist) {
    own_hist.resize((size_t)std::max(0, max_cycles) + 1);
    hist = own_hist.data();
  }
  double r0, l2, l2F = c->f_l2;
  c->l2_hist.clear();
  c->step_cycles.clear();
  L0.X[0] = c->x0;
  L0.b = const_cast<double*>(b);
  L0.cur = 0;
  c->u_cur = 0;
  launch_box_copy(c, c->x0, warm ? x : nullptr);
  int rc;
  if (bnorm < 0.0) {
    launch_residual_norm(c, b, c->zero, nullptr);
    rc = read_norm(c, bnorm, l2F);
    if (rc) return rc;
  }
  l2 = l2F;  // u = 0: the residual is F
  if (mixed) {
    // r = F - A u, its float copy and the zero float start iterate
    launch_outer(c, c->x0, nullptr, nullptr, L0.b32, L0.X32[0]);
    rc = read_norm(c, r0, l2);
    if (rc) return rc;
  } else if (warm) {
    launch_residual_norm(c, b, c->x0, nullptr);
    rc = read_norm(c, r0, l2);
    if (rc) return rc;
  } else {
    r0 = bnorm;  // u = 0
  }
  if (hist) hist[0] = r0;
  c->l2_hist.push_back(l2);
  if (!mixed) gather_snap(c, 0, false);
  double prev = r0;
  int grow = 0, m = 0;
  bool conv = r0 <= rel_tol * bnorm;
  int status = MGFEM_OK;
  if (!std::isfinite(r0)) status = MGFEM_ERR_DIVERGED;
  const bool fused = !mixed && !reverse;  // norm of u_m from the first sweep of cycle m + 1
  bool first_done = false;
  // The mixed loop queues its next iteration before reading the norm it
  // waits for (when that iteration will most likely be needed): the outer
  // update writes the other float64 buffer, so the iterate whose norm is
  // pending survives it and the queued iteration can be discarded.  The
  // float64 forward cycle writes both level-0 buffers (a third buffer, which
  // would make it safe, pushed the level-0 vectors out of the last-level
  // cache and cost more than the launch gaps it saved) and the transposed
  // cycle smooths its incoming iterate in place, so they wait for every norm;
  // so do profiled solves, whose events are read per iteration.
  const bool ahead = mixed && !c->prof.on;
  struct Pending {
    double seq;          // the iteration's last reduction: the norm of `result`
    double* result;      // the iterate that norm belongs to
    const GraphEntry* g;
  };
  Pending pend[2];
  int queued = 0;
  double* result = c->x0;  // the iterate returned when the loop stops
  // The queue-ahead test with i norms read: the last factor applied once more
  // leaves the residual 4x above the target, so the iteration after the one
  // in flight will most likely be needed.
  auto would_queue = [&](int i) -> bool {
    const double rho = i > 0 ? hist[i] / std::max(hist[i - 1], 1e-300) : 1.0;
    return rel_tol <= 0.0 || hist[i] * rho > 4.0 * rel_tol * bnorm;
  };
  // Mixed precision: step j runs inner_cycles float32 cycles, or fewer where
  // the residuals say fewer reach the tolerance (so the last step does not
  // over-solve).  The count depends on the history alone, never on when the
  // loop reads it (a profiled solve reads every norm before it launches, an
  // unprofiled one queues ahead), so both run the same steps: a step that
  // would be queued ahead runs the full count; any other is launched after
  // the norm of the step before it has been read and runs as many cycles as
  // the factor per float32 cycle of that step needs to bring that norm to the
  // target, rounded up.  The first step's factor is not used: its first
  // cycles converge much faster than the later ones.
  const int K = mixed ? c->p.inner_cycles : 1;
  std::vector<int> step_inner;  // float32 cycles of each launched step
  const char* fi_env = std::getenv("MGFEM_FIXED_INNER");
  const bool adapt = mixed && K > 1 && rel_tol > 0.0 && !(fi_env && fi_env[0] && fi_env[0] != '0');
  auto inner_for = [&](int j) -> int {  // step j = 1, 2, ...
    if (!adapt || j < 3 || would_queue(j - 2) || m != j - 1) return K;
    const double r = hist[j - 1], rp = hist[j - 2];
    const int kp = step_inner[j - 2];
    if (!(r > 0.0) || !(rp > r) || kp < 1) return K;
    const double rho = std::pow(r / rp, 1.0 / kp);
    const double need = std::log(rel_tol * bnorm / r) / std::log(rho);
    if (!std::isfinite(need)) return K;
    return std::max(1, std::min(K, (int)std::ceil(need)));
  };
  auto launch = [&](Pending& out) -> int {
    const GraphEntry* g = nullptr;
    const int inner = inner_for((int)step_inner.size() + 1);
    const int e = run_iteration(c, IterKind{mixed, reverse, first_done, inner}, &g);
    if (e) return e;
    step_inner.push_back(inner);
    first_done = fused;
    out.seq = c->red_seq;
    out.g = g;
    // fused: the closing sweep read the next iterate and wrote the other buffer
    out.result = mixed ? L0.X[c->u_cur] : fused ? L0.X[1 - L0.cur] : L0.X[L0.cur];
    return MGFEM_OK;
  };
  if (status == MGFEM_OK && !conv && m < max_cycles) {
    rc = launch(pend[0]);
    if (rc) return rc;
    queued = 1;
  }
  while (queued > 0) {
    // queue the next iteration now when it will most likely be needed
    if (ahead && queued == 1 && m + 1 < max_cycles && would_queue(m)) {
      rc = launch(pend[1]);
      if (rc) return rc;
      queued = 2;
    }
    double rm;
    rc = read_norm(c, rm, l2, nullptr, pend[0].seq);
    if (rc) return rc;
    if (pend[0].g && c->prof.on) {
      rc = prof_collect_graph(c, *pend[0].g);
      if (rc) return rc;
    }
    result = pend[0].result;
    pend[0] = pend[1];
    --queued;
    ++m;
    if (hist) hist[m] = rm;
    c->l2_hist.push_back(l2);
    if (!std::isfinite(rm)) {
      status = MGFEM_ERR_DIVERGED;
      break;
    }
    grow = rm > prev ? grow + 1 : 0;
    if (grow >= 3) {
      status = MGFEM_ERR_DIVERGED;
      break;
    }
    prev = rm;
    conv = rm <= rel_tol * bnorm;
    if (conv) break;
    if (queued == 0 && m < max_cycles) {
      rc = launch(pend[0]);
      if (rc) return rc;
      queued = 1;
    }
  }
  // an iteration still queued is discarded: it never writes `result` (the
  // export below is ordered after it on the stream)
  c->step_cycles.assign(step_inner.begin(), step_inner.begin() + std::min<size_t>(m, step_inner.size()));
  launch_export(c, x, result);
  MGFEM_HIP_TRY(hipGetLastError());
  MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  prof_collect(c);
  L0.b = nullptr;
  L0.cur = 0;
  c->u_cur = 0;
  if (ncyc) *ncyc = m;
  if (status != MGFEM_OK) {
    c->last_error = "residual not finite or growing";
    return status;
  }
  if (!conv && rel_tol > 0.0) {
    c->last_error = "tolerance not reached within max_cycles";
    return MGFEM_ERR_NOT_CONVERGED;
  }
  return MGFEM_OK;
}

// Largest eigenvalue and the last component of its unit eigenvector for the
// symmetric tridiagonal matrix with diagonal a and off-diagonal b: bisection
// on the Sturm count, then two steps of inverse iteration with the factorised
// (theta' I - T), positive definite for theta' just above the top eigenvalue.
void top_ritz(const std::vector<double>& a, const std::vector<double>& b, double& theta, double& ylast) {
  const int m = (int)a.size();
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_above = [&](double x) {  // eigenvalues > x
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
      d = (a[i] - x) - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d > 0.0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(hi), std::fabs(lo)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_above(mid) >= 1) lo = mid;
    else hi = mid;
  }
  theta = hi;
  const double sh = hi + 1e-13 * std::max(1.0, std::fabs(hi));
  std::vector<double> dg(m), y(m, 1.0);
  for (int rep = 0; rep < 2; ++rep) {
    // (sh I - T) z = y by the L D L^T recurrence of a tridiagonal matrix
    std::vector<double> l(m, 0.0), z(m);
    dg[0] = sh - a[0];
    for (int i = 1; i < m; ++i) {
      l[i] = -b[i - 1] / dg[i - 1];
      dg[i] = (sh - a[i]) - l[i] * (-b[i - 1]);
    }
    z[0] = y[0];
    for (int i = 1; i < m; ++i) z[i] = y[i] - l[i] * z[i - 1];
    for (int i = 0; i < m; ++i) z[i] /= dg[i];
    for (int i = m - 2; i >= 0; --i) z[i] -= l[i + 1] * z[i + 1];
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += z[i] * z[i];
    nrm = std::sqrt(nrm);
    for (int i = 0; i < m; ++i) y[i] = z[i] / nrm;
  }
  ylast = y[m - 1];
}

// C of the global generalised eigenproblem K v = Lambda S v (section 5.2) by
// the Lanczos iteration for S^-1 K in the S inner product.  S is the cut
// stiffness of a second context (kOpStiffness) whose multigrid solves give
// S^-1; K (over the Dirichlet segments) is applied from its gathered rows.
// Both vanish on the constants, so every iterate is kept free of them (mean
// over the active nodes removed); the diagonal scaling of the stored rows of
// S by 1 + 1e-12 that keeps the coarsest factor positive changes C by a
// relative 1e-12 times the ratio of the diagonal to the quadratic form of S
// on the top eigenvector.  Stops when the Ritz residual of the top Ritz value
// falls below 1e-11 of it, or after 400 steps.
int global_constant(const double* psi, const double* chi, int32_t N, const mgfem_params& p, void* stream,
                    double* C_out, int* iters_out) {
  mgfem_params ps = p;
  ps.stab_rule = MGFEM_STAB_FIXED;
  ps.lambda_fixed = 1.0;
  ps.precision = MGFEM_PREC_FP64;
  ps.cycle = MGFEM_CYCLE_V;
  ps.coarse_op = MGFEM_COARSE_GALERKIN;
  mgfem_ctx* s = nullptr;
  int rc = setup_impl(psi, chi, N, &ps, stream, &s, kOpStiffness);
  if (rc != MGFEM_OK) return fail(nullptr, rc, "global stabilisation: " + g_setup_error);
  struct Owner {
    mgfem_ctx* s;
    ~Owner() { free_ctx(s); }
  } owner{s};
  auto bail = [&](int code) { return fail(nullptr, code, "global stabilisation: " + s->last_error); };
  const int64_t n = s->lv[0].n;
  double *q = nullptr, *qp = nullptr, *w = nullptr, *u = nullptr, *sw = nullptr, *ones = nullptr;
  for (double** v : {&q, &qp, &w, &u, &sw, &ones})
    if (ctx_alloc_t(s, v, n) != hipSuccess) return fail(nullptr, MGFEM_ERR_OOM, "global stabilisation: allocation");
  launch_active_ones(s, ones);
  const double nact = (double)s->info.n_active;
  auto dot = [&](const double* x, const double* y, double& out) {
    launch_dot_reduce(s, x, y);
    double mx, l2;
    return read_norm(s, mx, l2, &out);
  };
  auto project = [&](double* x) {  // remove the mean over the active nodes
    double sum = 0.0;
    const int r = dot(x, ones, sum);
    if (r == MGFEM_OK) launch_shift_active(s, x, sum / nact);
    return r;
  };
  auto snorm2 = [&](const double* x, double& out) {  // x^T S x (sw = -S x)
    launch_residual_norm(s, s->zero, x, sw);
    double t = 0.0;
    const int r = dot(x, sw, t);
    out = -t;
    return r;
  };
  launch_start_vector(s, w);
  if ((rc = project(w)) || (rc = snorm2(w, *C_out))) return bail(rc);
  double nn = *C_out;
  *C_out = 0.0;
  *iters_out = 0;
  if (!(nn > 0.0)) return MGFEM_OK;
  launch_scale(s, q, w, 1.0 / std::sqrt(nn));
  launch_zero(s, qp, n);
  std::vector<double> al, be, hist(61);
  double beta = 0.0, theta = 0.0, ylast = 1.0;
  const int max_steps = (int)std::min<int64_t>(400, s->info.n_active);
  for (int j = 0; j < max_steps; ++j) {
    double a = 0.0;
    launch_k_apply(s, q, u);  // u = K q
    if ((rc = dot(q, u, a))) return bail(rc);
    launch_copy(s, s->F, u, n);
    int nc = 0;
    rc = iterate(s, w, s->F, 1e-12, 60, false, false, false, -1.0, hist.data(), &nc);  // w = S^-1 u
    if (rc != MGFEM_OK && !(nc > 0 && hist[nc] <= 1e-10 * hist[0])) return bail(rc);
    if ((rc = project(w))) return bail(rc);
    launch_lanczos_update(s, w, q, qp, a, beta);
    double bb = 0.0;
    if ((rc = snorm2(w, bb))) return bail(rc);
    al.push_back(a);
    top_ritz(al, be, theta, ylast);
    beta = std::sqrt(std::max(bb, 0.0));
    *iters_out = j + 1;
    if (beta * std::fabs(ylast) <= 1e-11 * std::fabs(theta) || beta <= 1e-14 * std::fabs(theta)) break;
    be.push_back(beta);
    std::swap(qp, q);
    launch_scale(s, q, w, 1.0 / beta);
  }
  *C_out = theta;
  hipError_t e = hipStreamSynchronize(s->s);
  if (e != hipSuccess) return fail(nullptr, MGFEM_ERR_HIP, "global stabilisation: stream error");
  return MGFEM_OK;
}

// The calls of one problem need a handle made by mgfem_setup or
// mgfem_setup_mixed_bc: a batched handle has no levels of its own (its
// problems live in member contexts), and a member context is reached only
// through mgfem_solve_batched.
int single_problem_check(mgfem_ctx* c) {
  if (!c) return MGFEM_ERR_INVALID_ARG;
  if (c->batched_member || !c->members.empty() || c->lv.empty())
    return fail(c, MGFEM_ERR_INVALID_ARG, "batched handle: use mgfem_solve_batched");
  return MGFEM_OK;
}

}  // namespace

extern "C" {

int mgfem_solve(mgfem_handle c, const double* f_dev, const double* g_dev, double rel_tol,
                int32_t max_cycles, uint32_t flags, double* u_dev, double* res_hist_host,
                int32_t* n_cycles) {
  return mgfem_solve_mixed_bc(c, f_dev, g_dev, nullptr, rel_tol, max_cycles, flags, u_dev, res_hist_host,
                              n_cycles);
}

int mgfem_solve_mixed_bc(mgfem_handle c, const double* f_dev, const double* gD_dev, const double* gN_dev,
                         double rel_tol, int32_t max_cycles, uint32_t flags, double* u_dev,
                         double* res_hist_host, int32_t* n_cycles) {
  const double* g_dev = gD_dev;
  if (const int e = single_problem_check(c)) return e;
  if (!f_dev || !g_dev || !u_dev || max_cycles < 0)
    return fail(c, MGFEM_ERR_INVALID_ARG, "f, g and u must be device pointers; max_cycles >= 0");
  const bool warm = (flags & MGFEM_SOLVE_WARM_START) != 0;
  if (warm) launch_mask_inactive(c, u_dev);
  launch_rhs(c, f_dev, g_dev, gN_dev, c->F);
  MGFEM_HIP_TRY(hipGetLastError());
  double bnorm, l2;
  int rc = read_norm(c, bnorm, l2);
  if (rc) return rc;
  c->f_l2 = l2;
  int nc = 0;
  rc = iterate(c, u_dev, c->F, rel_tol, max_cycles, false, c->p.precision == MGFEM_PREC_MIXED, warm, bnorm,
               res_hist_host, &nc);
  if (n_cycles) *n_cycles = nc;
  return rc;
}

int mgfem_adjoint(mgfem_handle c, const double* dJdu_dev, double rel_tol, int32_t max_cycles,
                  double* lam_dev, double* dJdf_dev, double* dJdg_dev, double* res_hist_host,
                  int32_t* n_cycles) {
  if (const int e = single_problem_check(c)) return e;
  if (!dJdu_dev || max_cycles < 0) return fail(c, MGFEM_ERR_INVALID_ARG, "dJdu must be a device pointer");
  double* lam = lam_dev ? lam_dev : c->lam;
  // the adjoint right-hand side must vanish off the active nodes
  launch_sub_active(c, c->F, dJdu_dev, c->zero);
  MGFEM_HIP_TRY(hipGetLastError());
  int nc = 0;
  int rc = iterate(c, lam, c->F, rel_tol, max_cycles, true, false, false, -1.0, res_hist_host, &nc);
  if (n_cycles) *n_cycles = nc;
  if (rc != MGFEM_OK && rc != MGFEM_ERR_NOT_CONVERGED) return rc;
  if (dJdf_dev) launch_mass_apply(c, lam, dJdf_dev);
  if (dJdg_dev) launch_gt_apply(c, lam, dJdg_dev);
  MGFEM_HIP_TRY(hipGetLastError());
  MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  return rc;
}

int mgfem_adjoint_neumann(mgfem_handle c, const double* lam_dev, double* dJdgN_dev) {
  if (const int e = single_problem_check(c)) return e;
  if (!lam_dev || !dJdgN_dev) return fail(c, MGFEM_ERR_INVALID_ARG, "lam and dJdgN must be device pointers");
  launch_gn_apply(c, lam_dev, dJdgN_dev);  // GN^T = GN
  MGFEM_HIP_TRY(hipGetLastError());
  MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  return MGFEM_OK;
}

int mgfem_misfit(mgfem_handle c, const double* u_dev, const double* ut_dev, double* J_host,
                 double* dJdu_dev) {
  if (const int e = single_problem_check(c)) return e;
  if (!u_dev || !ut_dev || !J_host) return fail(c, MGFEM_ERR_INVALID_ARG, "u, ut and J must be given");
  double* e = c->F64tmp;
  double* Me = dJdu_dev ? dJdu_dev : c->lam;
  launch_sub_active(c, e, u_dev, ut_dev);
  launch_mass_apply(c, e, Me);
  launch_dot_reduce(c, e, Me);
  MGFEM_HIP_TRY(hipGetLastError());
  double mx, l2, sum;
  int rc = read_norm(c, mx, l2, &sum);
  if (rc) return rc;
  *J_host = 0.5 * sum;
  return MGFEM_OK;
}

int mgfem_smooth(mgfem_handle c, int32_t level, double* x_dev, const double* b_dev, int32_t steps,
                 int32_t reverse) {
  if (!c || level < 0 || level + 1 >= (int)c->lv.size() || !x_dev || !b_dev || steps < 0)
    return c ? fail(c, MGFEM_ERR_INVALID_ARG, "bad level (the coarsest has no smoother) or pointer")
             : MGFEM_ERR_INVALID_ARG;
  Level& L = c->lv[level];
  double* sx = L.X[0];
  double* sb = L.b;
  L.X[0] = x_dev;
  L.b = const_cast<double*>(b_dev);
  L.cur = 0;
  gather_snap(c, level, false);
  for (int s = 0; s < steps; ++s) smooth_level(c, level, reverse != 0, false);
  if (L.cur == 1) launch_copy(c, x_dev, L.X[1], L.n);
  L.X[0] = sx;
  L.b = sb;
  L.cur = 0;
  MGFEM_HIP_TRY(hipGetLastError());
  MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  return MGFEM_OK;
}

int mgfem_residual_l2(mgfem_handle c, double* l2_hist_host, int32_t capacity, int32_t* count) {
  if (!c || capacity < 0 || (capacity > 0 && !l2_hist_host)) return MGFEM_ERR_INVALID_ARG;
  const int n = std::min(capacity, (int)c->l2_hist.size());
  for (int m = 0; m < n; ++m) l2_hist_host[m] = c->l2_hist[m];
  if (count) *count = (int32_t)c->l2_hist.size();
  return MGFEM_OK;
}

int mgfem_step_cycles(mgfem_handle c, int32_t* cycles_host, int32_t capacity, int32_t* count) {
  if (!c || capacity < 0 || (capacity > 0 && !cycles_host)) return MGFEM_ERR_INVALID_ARG;
  const int n = std::min(capacity, (int)c->step_cycles.size());
  for (int m = 0; m < n; ++m) cycles_host[m] = c->step_cycles[m];
  if (count) *count = (int32_t)c->step_cycles.size();
  return MGFEM_OK;
}

int mgfem_level_counts(mgfem_handle c, int32_t level, int64_t* n_active, int64_t* n_stored,
                       int64_t* n_cut) {
  if (!c || level < 0 || level >= (int)c->lv.size()) return MGFEM_ERR_INVALID_ARG;
  const Level& L = c->lv[level];
  if (n_active) *n_active = L.n_active;
  if (n_stored) *n_stored = L.n_stored;
  if (n_cut) *n_cut = L.cut_off[4];
  return MGFEM_OK;
}

int mgfem_profile(mgfem_handle c, int32_t enable) {
  if (!c || enable < 0 || enable > 1000) return MGFEM_ERR_INVALID_ARG;
  c->prof.on = enable != 0;
  c->prof.repeat = enable > 1 ? enable : 1;
  for (int k = 0; k < 4; ++k) {
    c->prof.launches[k] = 0;
    c->prof.ms[k] = 0.0;
    c->prof.bytes[k] = 0.0;
  }
  return MGFEM_OK;
}

int mgfem_profile_read(mgfem_handle c, int32_t kernel_class, int64_t* launches, double* total_ms,
                       double* alg_bytes) {
  if (!c || kernel_class < 0 || kernel_class > 3) return MGFEM_ERR_INVALID_ARG;
  if (launches) *launches = c->prof.launches[kernel_class];
  if (total_ms) *total_ms = c->prof.ms[kernel_class];
  if (alg_bytes) *alg_bytes = c->prof.bytes[kernel_class];
  return MGFEM_OK;
}

int mgfem_export(mgfem_handle c, int32_t what, int32_t level, double* dst) {
  if (!c || !dst || level < 0 || level >= (int)c->lv.size()) return MGFEM_ERR_INVALID_ARG;
  Level& L = c->lv[level];
  const int64_t n = L.n, nc = (int64_t)c->N * c->N;
  const bool l0 = level == 0;
  switch (what) {
    case MGFEM_EXPORT_PSI:
      if (!l0) return fail(c, MGFEM_ERR_INVALID_ARG, "level 0 only");
      launch_copy(c, dst, c->psi, n);
      break;
    case MGFEM_EXPORT_CELL_TYPE:
      if (!l0) return fail(c, MGFEM_ERR_INVALID_ARG, "level 0 only");
      launch_u8_to_f64(c, c->cell_type, dst, nc);
      break;
    case MGFEM_EXPORT_CELL_LAMBDA:
      if (!l0) return fail(c, MGFEM_ERR_INVALID_ARG, "level 0 only");
      launch_copy(c, dst, c->cell_lambda, nc);
      break;
    case MGFEM_EXPORT_A: launch_copy(c, dst, L.A, 9 * n); break;
    case MGFEM_EXPORT_M:
      if (!l0) return fail(c, MGFEM_ERR_INVALID_ARG, "level 0 only");
      launch_copy(c, dst, c->M, 9 * n);
      break;
    case MGFEM_EXPORT_G:
      if (!l0) return fail(c, MGFEM_ERR_INVALID_ARG, "level 0 only");
      launch_copy(c, dst, c->G, 9 * n);
      break;
    case MGFEM_EXPORT_GN:
      if (!l0) return fail(c, MGFEM_ERR_INVALID_ARG, "level 0 only");
      if (c->GN) launch_copy(c, dst, c->GN, 9 * n);
      else launch_zero(c, dst, 9 * n);
      break;
    case MGFEM_EXPORT_NODE_FLAGS: launch_u8_to_f64(c, L.flags, dst, n); break;
    case MGFEM_EXPORT_RHS:
      if (!l0) return fail(c, MGFEM_ERR_INVALID_ARG, "level 0 only");
      launch_copy(c, dst, c->F, n);
      break;
    default: return fail(c, MGFEM_ERR_INVALID_ARG, "unknown export");
  }
  MGFEM_HIP_TRY(hipGetLastError());
  MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  return MGFEM_OK;
}

}  // extern "C"
