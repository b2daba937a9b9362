// Batched solves on the tiled kernels (host side).
//
// All problems of a batch advance through the same sequence of steps: the
// float64 outer defect-correction step on level 0, then one float32 V-cycle
// from zero on its residual, level by level.  Each step is one launch whose
// workgroups take (problem, unit) items of a work list: the sweep tiles, cut
// groups and residual-restriction tiles of level d of every problem that
// smooths level d, the row blocks of the coarse maps of the problems whose
// coarse part starts at level d + 1, the box blocks of level 0.  A problem
// leaves the lists once its residual meets the tolerance (or it diverges or
// runs out of cycles), so later launches carry only the problems still
// iterating.  A problem's steps are those of the single-problem mixed
// solve (the same kernels), so its iterates are the same.
//
// Ping-pong parities: every problem that smooths level d has run the same
// steps on it since the solve began, so one parity per level serves them
// all; a problem whose coarse part starts at level d + 1 reads that level's
// iterate from buffer 0, where its coarse map writes it.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "mgfem_internal.h"

namespace mgfem {

struct TeamPlan {
  bool ok = false;
  int P = 0;
  int depth = 0;                     // largest first coarse level over the members
  std::vector<int> lc;               // first coarse level per member
  std::vector<void*> tab[4];         // per float-cycle kind: one device table of P entries per level
  int cut_lds = 0, map_lds = 0;      // dynamic LDS of the cut and map launches
  std::vector<TeamL0> l0h;           // level-0 entries (host copy)
  TeamL0* l0 = nullptr;              // device copy
  int2* work = nullptr;              // device work lists of the current active set
  size_t work_cap = 0;
  int* probs = nullptr;              // device: the active problems (reductions)
  double* red = nullptr;             // device: (max, sum of squares) per problem
  double* red_host = nullptr;        // pinned copy
  // segments of the work buffer: float-cycle kinds [kind][level], level-0 kinds
  std::vector<int> seg_off, seg_cnt;
  int l0_off[5] = {0, 0, 0, 0, 0}, l0_cnt[5] = {0, 0, 0, 0, 0};
  int nprobs = 0;
};

namespace {

int seg(const TeamPlan& T, int kind, int d) { return kind * T.depth + d; }

// work lists of the active problems (all float-cycle and level-0 kinds)
int team_lists(mgfem_ctx* b, TeamPlan& T, const std::vector<int>& active, bool with_export) {
  mgfem_ctx* c = b;
  std::vector<int2> w;
  T.seg_off.assign(4 * T.depth, 0);
  T.seg_cnt.assign(4 * T.depth, 0);
  for (int kind = 0; kind < 4; ++kind)
    for (int d = 0; d < T.depth; ++d) {
      T.seg_off[seg(T, kind, d)] = (int)w.size();
      for (int p : active) {
        mgfem_ctx* m = b->members[p];
        const bool smooths = d < T.lc[p];
        const bool maps = T.lc[p] == d + 1;
        if ((kind == kTeamMap && !maps) || (kind != kTeamMap && !smooths)) continue;
        const int u = team_units(m, kind, d);
        for (int q = 0; q < u; ++q) w.push_back(make_int2(p, q));
      }
      T.seg_cnt[seg(T, kind, d)] = (int)w.size() - T.seg_off[seg(T, kind, d)];
    }
  for (int kind = 0; kind < 5; ++kind) {
    T.l0_off[kind] = (int)w.size();
    if (kind != kTeamExport || with_export) {
      const std::vector<int>& who = active;
      for (int p : who) {
        const int u = team_l0_units(T.l0h[p], kind);
        for (int q = 0; q < u; ++q) w.push_back(make_int2(p, q));
      }
    }
    T.l0_cnt[kind] = (int)w.size() - T.l0_off[kind];
  }
  if (w.size() > T.work_cap) {
    T.work_cap = std::max(w.size(), 2 * T.work_cap);
    MGFEM_HIP_TRY(ctx_alloc_t(b, &T.work, T.work_cap));
  }
  if (!w.empty())
    MGFEM_HIP_TRY(hipMemcpyAsync(T.work, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice, b->s));
  T.nprobs = (int)active.size();
  if (!active.empty())
    MGFEM_HIP_TRY(hipMemcpyAsync(T.probs, active.data(), active.size() * sizeof(int), hipMemcpyHostToDevice, b->s));
  // the host vectors must outlive the copies
  MGFEM_HIP_TRY(hipStreamSynchronize(b->s));
  return MGFEM_OK;
}

void launch_kind(mgfem_ctx* b, TeamPlan& T, int kind, int d, int par, int parc, int prolong) {
  const int k = seg(T, kind, d);
  const int lds = kind == kTeamCut ? T.cut_lds : kind == kTeamMap ? T.map_lds : 0;
  team_launch(b->s, kind, T.tab[kind][d], T.work + T.seg_off[k], T.seg_cnt[k], par, parc, prolong, lds);
}

void launch_l0(mgfem_ctx* b, TeamPlan& T, int kind, int upar, int epar) {
  team_l0_launch(b->s, kind, T.l0, T.work + T.l0_off[kind], T.l0_cnt[kind], upar, epar);
}

// one float V-cycle from level d down, for the problems in the lists;
// par[l]: which buffer holds level l's iterate
void team_level(mgfem_ctx* b, TeamPlan& T, int d, std::vector<int>& par) {
  const int nu1 = b->p.nu1, nu2 = b->p.nu2;
  for (int s = 0; s < nu1; ++s) {
    launch_kind(b, T, kTeamSweep, d, par[d], 0, 0);
    par[d] ^= 1;
    launch_kind(b, T, kTeamCut, d, par[d], 0, 0);
  }
  launch_kind(b, T, kTeamRR, d, par[d], par[d + 1], 0);
  launch_kind(b, T, kTeamMap, d, 0, 0, 0);
  if (d + 1 < T.depth) team_level(b, T, d + 1, par);
  launch_kind(b, T, kTeamSweep, d, par[d], par[d + 1], 1);  // x + P x_c, then the sweep
  par[d] ^= 1;
  launch_kind(b, T, kTeamCut, d, par[d], 0, 0);
  for (int s = 1; s < nu2; ++s) {
    launch_kind(b, T, kTeamSweep, d, par[d], 0, 0);
    par[d] ^= 1;
    launch_kind(b, T, kTeamCut, d, par[d], 0, 0);
  }
}

int read_red(mgfem_ctx* b, TeamPlan& T) {
  mgfem_ctx* c = b;
  team_reduce(b->s, T.l0, T.probs, T.nprobs, T.red);
  MGFEM_HIP_TRY(hipMemcpyAsync(T.red_host, T.red, 2 * T.P * sizeof(double), hipMemcpyDeviceToHost, b->s));
  MGFEM_HIP_TRY(hipStreamSynchronize(b->s));
  return MGFEM_OK;
}

}  // namespace

bool team_ok(const mgfem_ctx* b) { return b->team && b->team->ok; }

void team_free(mgfem_ctx* b) {
  if (!b->team) return;
  if (b->team->red_host) (void)hipHostFree(b->team->red_host);
  delete b->team;  // device buffers are the handle's allocations
  b->team = nullptr;
}

// Tables of a batched handle whose members (set up in mixed precision) can
// all take the tiled path: every smoothed level with the small tile shapes,
// cut groups where there are cut vertices, a float coarse map, nu2 >= 1.
int team_build(mgfem_ctx* b) {
  mgfem_ctx* c = b;
  TeamPlan* T = new TeamPlan();
  b->team = T;
  const int P = (int)b->members.size();
  T->P = P;
  T->lc.resize(P);
  bool ok = P > 0 && b->p.nu2 >= 1;
  for (int p = 0; p < P && ok; ++p) {
    mgfem_ctx* m = b->members[p];
    const int lc = m->cplan.lc;
    T->lc[p] = lc;
    ok = lc >= 1 && team_units(m, kTeamMap, 0) > 0;
    for (int l = 0; l < lc && ok; ++l)
      for (int kind : {kTeamSweep, kTeamCut, kTeamRR})
        if (team_units(m, kind, l) < 0) ok = false;
    if (ok) T->depth = std::max(T->depth, lc);
  }
  if (!ok) return MGFEM_OK;  // the persistent kernel serves this batch
  for (int kind = 0; kind < 4; ++kind) {
    const size_t eb = team_entry_bytes(kind);
    for (int d = 0; d < T->depth; ++d) {
      std::vector<unsigned char> host((size_t)P * eb, 0);
      for (int p = 0; p < P; ++p) {
        mgfem_ctx* m = b->members[p];
        const bool use = kind == kTeamMap ? T->lc[p] == d + 1 : d < T->lc[p];
        if (!use) continue;
        team_entry(m, kind, d, host.data() + (size_t)p * eb);
        if (kind == kTeamCut) T->cut_lds = std::max(T->cut_lds, team_lds(m, kind, d));
        if (kind == kTeamMap) T->map_lds = std::max(T->map_lds, team_lds(m, kind, d));
      }
      void* dev = nullptr;
      MGFEM_HIP_TRY(ctx_alloc(b, &dev, host.size()));
      MGFEM_HIP_TRY(hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, b->s));
      MGFEM_HIP_TRY(hipStreamSynchronize(b->s));
      T->tab[kind].push_back(dev);
    }
  }
  T->l0h.resize(P);
  for (int p = 0; p < P; ++p) team_l0_entry(b->members[p], &T->l0h[p]);
  MGFEM_HIP_TRY(ctx_alloc_t(b, &T->l0, P));
  MGFEM_HIP_TRY(ctx_alloc_t(b, &T->probs, P));
  MGFEM_HIP_TRY(ctx_alloc_t(b, &T->red, 2 * P));
  MGFEM_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&T->red_host), 2 * P * sizeof(double)));
  T->ok = true;
  return MGFEM_OK;
}

// One batched solve on the tiled path.  hist: count x (max_cycles + 1), ncyc: count.
int team_solve(mgfem_ctx* b, const double* const* f, const double* const* g, double* const* u, double rel_tol,
               int max_cycles, std::vector<double>& hist, std::vector<int>& ncyc, float* ms_out) {
  mgfem_ctx* c = b;
  TeamPlan& T = *b->team;
  const int P = T.P, H = max_cycles + 1;
  hist.assign((size_t)P * H, 0.0);
  ncyc.assign(P, 0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MGFEM_HIP_TRY(hipEventCreate(&e0));
  MGFEM_HIP_TRY(hipEventCreate(&e1));
  MGFEM_HIP_TRY(hipEventRecord(e0, b->s));
  for (int p = 0; p < P; ++p) {
    T.l0h[p].f = f[p];
    T.l0h[p].g = g[p];
    T.l0h[p].u_out = u[p];
    T.l0h[p].ucur = 0;
  }
  MGFEM_HIP_TRY(hipMemcpyAsync(T.l0, T.l0h.data(), P * sizeof(TeamL0), hipMemcpyHostToDevice, b->s));
  std::vector<int> active(P);
  for (int p = 0; p < P; ++p) active[p] = p;
  int rc = team_lists(b, T, active, false);
  if (rc) return rc;
  // F = M f + G g and its norm
  launch_l0(b, T, kTeamCutRows, 0, 0);
  launch_l0(b, T, kTeamRhs, 0, 0);
  if ((rc = read_red(b, T))) return rc;
  std::vector<double> bnorm(P), prev(P);
  std::vector<int> grow(P, 0);
  for (int p = 0; p < P; ++p) bnorm[p] = T.red_host[2 * p];
  // u = 0: r = F
  launch_l0(b, T, kTeamOuterFirst, 0, 0);
  if ((rc = read_red(b, T))) return rc;
  std::vector<int> ucur(P, 0);
  auto done = [&](int p, double r) {
    if (!std::isfinite(r)) return true;
    return rel_tol > 0.0 && r <= rel_tol * bnorm[p];
  };
  std::vector<int> next;
  for (int p : active) {
    const double r = T.red_host[2 * p];
    hist[(size_t)p * H] = r;
    prev[p] = r;
    if (!done(p, r) && max_cycles > 0) next.push_back(p);
  }
  std::vector<int> par(T.depth + 1, 0);
  int upar = 0;
  int m = 0;
  bool changed = next.size() != active.size();
  active.swap(next);
  // Float32 cycles of each step: inner_cycles, or fewer when every problem
  // still iterating would run fewer in its own mixed-precision solve, by the
  // single-problem rule: a problem whose last factor, applied once more,
  // still leaves it 4x above its target, and any problem in its first two
  // steps, needs the full count; any other needs the number of its last
  // step's factors per float32 cycle that brings its residual to the target.
  // All problems of a step share one count (their cycles share launches).
  const int K = b->p.inner_cycles;
  const char* fi_env = std::getenv("MGFEM_FIXED_INNER");
  const bool adapt = K > 1 && rel_tol > 0.0 && !(fi_env && fi_env[0] && fi_env[0] != '0');
  std::vector<int> step_k;  // float32 cycles of each step
  auto need = [&](int p, int j) -> int {  // step j = m + 1 of problem p
    const double* h = hist.data() + (size_t)p * H;
    if (j < 3) return K;
    const double rq = h[j - 3] > 0.0 ? h[j - 2] / h[j - 3] : 1.0;
    if (h[j - 2] * rq > 4.0 * rel_tol * bnorm[p]) return K;
    const double r = h[j - 1], rp = h[j - 2];
    const int kp = step_k[j - 2];
    if (!(r > 0.0) || !(rp > r) || kp < 1) return K;
    const double rho = std::pow(r / rp, 1.0 / kp);
    const double n = std::log(rel_tol * bnorm[p] / r) / std::log(rho);
    if (!std::isfinite(n)) return K;
    return std::max(1, std::min(K, (int)std::ceil(n)));
  };
  while (!active.empty() && m < max_cycles) {
    if (changed && (rc = team_lists(b, T, active, false))) return rc;
    int kstep = adapt ? 1 : K;
    if (adapt)
      for (int p : active) kstep = std::max(kstep, need(p, m + 1));
    step_k.push_back(kstep);
    for (int q = 0; q < kstep; ++q) team_level(b, T, 0, par);
    const int ce = par[0];
    launch_l0(b, T, kTeamOuter, upar, ce);
    upar ^= 1;
    par[0] = 1 - ce;
    ++m;
    if ((rc = read_red(b, T))) return rc;
    next.clear();
    for (int p : active) {
      const double r = T.red_host[2 * p];
      hist[(size_t)p * H + m] = r;
      ncyc[p] = m;
      ucur[p] = upar;
      grow[p] = r > prev[p] ? grow[p] + 1 : 0;
      prev[p] = r;
      if (!done(p, r) && grow[p] < 3 && m < max_cycles) next.push_back(p);
    }
    changed = next.size() != active.size();
    active.swap(next);
  }
  // every problem's result into the caller's arrays
  for (int p = 0; p < P; ++p) T.l0h[p].ucur = ucur[p];
  MGFEM_HIP_TRY(hipMemcpyAsync(T.l0, T.l0h.data(), P * sizeof(TeamL0), hipMemcpyHostToDevice, b->s));
  std::vector<int> all(P);
  for (int p = 0; p < P; ++p) all[p] = p;
  if ((rc = team_lists(b, T, all, true))) return rc;
  launch_l0(b, T, kTeamExport, 0, 0);
  MGFEM_HIP_TRY(hipGetLastError());
  MGFEM_HIP_TRY(hipEventRecord(e1, b->s));
  MGFEM_HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  MGFEM_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ms_out) *ms_out = ms;
  return MGFEM_OK;
}

}  // namespace mgfem
