// Setup, part 3 (host side of the runtime): launch plans built once per
// hierarchy from small device arrays copied back.
//
//  * Cut-vertex groups for the extra-smoothing kernel.  One smoothing step
//    applies 4 eta colour phases to the cut vertices; a value after them
//    depends on values at most 4 eta nodes away, so a group owning the cut
//    vertices of one tile and holding every cut vertex within 4 eta of that
//    tile (its closure) computes its own vertices exactly, alone.  Tiles
//    whose closure does not fit in LDS are split in four.
//  * The single-workgroup part: the coarsest levels whose arrays (iterate,
//    right-hand side, residual on the bounding box grown by one ring, the
//    stored stencil rows and the cut lists) fit in one workgroup's LDS.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <unordered_map>

#include "mgfem_internal.h"

namespace mgfem {
namespace {

inline int align16(int v) { return (v + 15) & ~15; }

__global__ void k_cutpos(const int* __restrict__ list, int cnt, int* __restrict__ pos) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < cnt) pos[list[q]] = q;
}

// closure-node coefficients in one contiguous record: 8 off-diagonals, 1/diagonal
__global__ void k_gather_coef(const double* __restrict__ A, int64_t n, const int* __restrict__ node, int cnt,
                              double* __restrict__ out, float* __restrict__ out32) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const int64_t k = node[t];
  const int pl[8] = {0, 1, 2, 3, 5, 6, 7, 8};
  for (int e = 0; e < 8; ++e) {
    const double v = A[pl[e] * n + k];
    out[9 * (int64_t)t + e] = v;
    if (out32) out32[9 * (int64_t)t + e] = (float)v;
  }
  const double d = A[4 * n + k];
  out[9 * (int64_t)t + 8] = 1.0 / d;
  if (out32) out32[9 * (int64_t)t + 8] = 1.0f / (float)d;
}

__global__ void k_fill_i(int* __restrict__ p, int64_t n, int v) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

struct GroupBuild {
  std::vector<int> info, node, q, ext;
  std::vector<uint8_t> own;
  std::vector<int16_t> nbr;
  int max_cl = 0, max_ext = 0, lds64 = 0, lds32 = 0;
};

// recursively split the rectangle [x0,x1) x [y0,y1) until each closure fits
bool build_groups(const std::vector<int>& nodes, const std::unordered_map<int, int>& cutq, int N, int D,
                  int x0, int x1, int y0, int y1, const std::vector<int>& owned_q, size_t lds_cap,
                  size_t tsize, GroupBuild& gb,
                  const std::vector<std::vector<int>>& buckets, int BT, int nbx, int nby) {
  if (owned_q.empty()) return true;
  const int s = N + 1;
  // closure: cut vertices in the rectangle grown by D
  std::vector<int> cl;
  const int bx0 = std::max(0, (x0 - D) / BT), bx1 = std::min(nbx - 1, (x1 - 1 + D) / BT);
  const int by0 = std::max(0, (y0 - D) / BT), by1 = std::min(nby - 1, (y1 - 1 + D) / BT);
  for (int by = by0; by <= by1; ++by)
    for (int bx = bx0; bx <= bx1; ++bx)
      for (int q : buckets[bx + by * nbx]) {
        const int k = nodes[q], i = k % s, j = k / s;
        if (i >= x0 - D && i < x1 + D && j >= y0 - D && j < y1 + D) cl.push_back(q);
      }
  // order: colour, then node index
  std::sort(cl.begin(), cl.end(), [&](int a, int b) {
    const int ka = nodes[a], kb = nodes[b];
    const int ca = (ka % s & 1) + 2 * (ka / s & 1), cb = (kb % s & 1) + 2 * (kb / s & 1);
    return ca != cb ? ca < cb : ka < kb;
  });
  std::unordered_map<int, int> local;
  local.reserve(cl.size() * 2);
  for (size_t t = 0; t < cl.size(); ++t) local[nodes[cl[t]]] = (int)t;
  std::unordered_map<int, int> extmap;
  std::vector<int> ext;
  std::vector<int16_t> nbr(8 * cl.size(), -1);
  const int pl[8] = {0, 1, 2, 3, 5, 6, 7, 8};
  for (size_t t = 0; t < cl.size(); ++t) {
    const int k = nodes[cl[t]], i = k % s, j = k / s;
    for (int e = 0; e < 8; ++e) {
      const int ii = i + pl[e] % 3 - 1, jj = j + pl[e] / 3 - 1;
      if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
      const int kk = ii + jj * s;
      auto it = local.find(kk);
      if (it != local.end()) {
        nbr[8 * t + e] = (int16_t)it->second;
        continue;
      }
      auto cq = cutq.find(kk);
      const int key = cq != cutq.end() ? -(1 + cq->second) : kk;
      auto ex = extmap.find(key);
      int idx;
      if (ex == extmap.end()) {
        idx = (int)ext.size();
        extmap[key] = idx;
        ext.push_back(key);
      } else {
        idx = ex->second;
      }
      nbr[8 * t + e] = (int16_t)(cl.size() + idx);
    }
  }
  const size_t bytes = (size_t)cut_lds_layout((int)cl.size(), (int)ext.size(), (int)tsize).total;
  if (bytes > lds_cap || cl.size() + ext.size() > 32000) {
    if (x1 - x0 <= 4 && y1 - y0 <= 4) return false;
    const int xm = (x0 + x1) / 2, ym = (y0 + y1) / 2;
    const int rx[4][2] = {{x0, xm}, {xm, x1}, {x0, xm}, {xm, x1}};
    const int ry[4][2] = {{y0, ym}, {y0, ym}, {ym, y1}, {ym, y1}};
    for (int h = 0; h < 4; ++h) {
      std::vector<int> sub;
      for (int q : owned_q) {
        const int k = nodes[q], i = k % s, j = k / s;
        if (i >= rx[h][0] && i < rx[h][1] && j >= ry[h][0] && j < ry[h][1]) sub.push_back(q);
      }
      if (!build_groups(nodes, cutq, N, D, rx[h][0], rx[h][1], ry[h][0], ry[h][1], sub, lds_cap, tsize,
                        gb, buckets, BT, nbx, nby))
        return false;
    }
    return true;
  }
  // colour offsets and ownership
  int col_off[5] = {0, 0, 0, 0, 0};
  for (size_t t = 0; t < cl.size(); ++t) {
    const int k = nodes[cl[t]];
    ++col_off[1 + (k % s & 1) + 2 * (k / s & 1)];
  }
  for (int cc = 1; cc < 5; ++cc) col_off[cc] += col_off[cc - 1];
  const int base = (int)gb.node.size(), ebase = (int)gb.ext.size();
  gb.info.push_back(base);
  gb.info.push_back((int)cl.size());
  gb.info.push_back(ebase);
  gb.info.push_back((int)ext.size());
  for (int cc = 0; cc < 5; ++cc) gb.info.push_back(col_off[cc]);
  for (size_t t = 0; t < cl.size(); ++t) {
    const int k = nodes[cl[t]], i = k % s, j = k / s;
    gb.node.push_back(k);
    gb.q.push_back(cl[t]);
    gb.own.push_back((i >= x0 && i < x1 && j >= y0 && j < y1) ? 1 : 0);
  }
  // neighbours outside the grid read the zero slot after the external values
  for (auto& r : nbr)
    if (r < 0) r = (int16_t)(cl.size() + ext.size());
  gb.nbr.insert(gb.nbr.end(), nbr.begin(), nbr.end());
  gb.lds64 = std::max(gb.lds64, cut_lds_layout((int)cl.size(), (int)ext.size(), 8).total);
  gb.lds32 = std::max(gb.lds32, cut_lds_layout((int)cl.size(), (int)ext.size(), 4).total);
  gb.ext.insert(gb.ext.end(), ext.begin(), ext.end());
  gb.max_cl = std::max(gb.max_cl, (int)cl.size());
  gb.max_ext = std::max(gb.max_ext, (int)ext.size());
  return true;
}

template <class V>
int upload(mgfem_ctx* c, V** dst, const std::vector<V>& src) {
  MGFEM_HIP_TRY(ctx_alloc_t(c, dst, std::max<size_t>(1, src.size())));
  if (!src.empty())
    MGFEM_HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice, c->s));
  return MGFEM_OK;
}

}  // namespace

int build_plans(mgfem_ctx* c) {
  const int nl = (int)c->lv.size();
  const bool mixed = c->p.precision == MGFEM_PREC_MIXED;
  int dev = 0;
  MGFEM_HIP_TRY(hipGetDevice(&dev));
  int lds_max = 65536;
  MGFEM_HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const size_t cap = (size_t)lds_max - 4096;  // room for the kernels' static LDS
  // --- cut positions, snapshots and cut groups, every level with smoothing
  const int D = 4 * c->p.eta;
  // MGFEM_NO_CUT_GROUPS=1: no group plans, so every level takes the list
  // smoother (the path of a level whose groups do not fit in LDS)
  const char* ng_env = std::getenv("MGFEM_NO_CUT_GROUPS");
  const bool no_groups = ng_env && ng_env[0] && ng_env[0] != '0';
  for (int l = 0; l + 1 < nl; ++l) {
    Level& L = c->lv[l];
    const int cnt = L.cut_off[4];
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.cutpos, L.n));
    hipLaunchKernelGGL(k_fill_i, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, c->s, L.cutpos, L.n, -1);
    if (cnt > 0)
      hipLaunchKernelGGL(k_cutpos, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, c->s, L.cut_list, cnt,
                         L.cutpos);
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.snap, std::max(1, cnt)));
    if (mixed) MGFEM_HIP_TRY(ctx_alloc_t(c, &L.snap32, std::max(1, cnt)));
    MGFEM_HIP_TRY(hipGetLastError());
    if (cnt == 0 || c->p.eta == 0 || no_groups) continue;
    std::vector<int> nodes(cnt);
    MGFEM_HIP_TRY(hipMemcpyAsync(nodes.data(), L.cut_list, cnt * sizeof(int), hipMemcpyDeviceToHost, c->s));
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
    std::unordered_map<int, int> cutq;
    cutq.reserve(cnt * 2);
    for (int q = 0; q < cnt; ++q) cutq[nodes[q]] = q;
    const int s = L.stride;
    const int BT = 16;
    const int nbx = (L.N + BT) / BT, nby = nbx;
    std::vector<std::vector<int>> buckets(nbx * nby);
    for (int q = 0; q < cnt; ++q) buckets[(nodes[q] % s) / BT + ((nodes[q] / s) / BT) * nbx].push_back(q);
    const int GT = 32;  // owned tile of one group
    const int ngx = (L.N + GT) / GT;
    std::vector<std::vector<int>> owned(ngx * ngx);
    for (int q = 0; q < cnt; ++q) owned[(nodes[q] % s) / GT + ((nodes[q] / s) / GT) * ngx].push_back(q);
    GroupBuild gb;
    bool ok = true;
    for (int g = 0; g < ngx * ngx && ok; ++g) {
      if (owned[g].empty()) continue;
      const int x0 = (g % ngx) * GT, y0 = (g / ngx) * GT;
      ok = build_groups(nodes, cutq, L.N, D, x0, x0 + GT, y0, y0 + GT, owned[g], cap, sizeof(double), gb,
                        buckets, BT, nbx, nby);
    }
    L.cp.ok = ok;
    if (!ok) continue;
    L.cp.ngroups = (int)gb.info.size() / 9;
    L.cp.max_cl = gb.max_cl;
    L.cp.max_ext = gb.max_ext;
    L.cp.lds64 = gb.lds64;
    L.cp.lds32 = gb.lds32;
    int rc;
    if ((rc = upload(c, &L.cp.g_info, gb.info))) return rc;
    if ((rc = upload(c, &L.cp.cl_node, gb.node))) return rc;
    if ((rc = upload(c, &L.cp.cl_q, gb.q))) return rc;
    if ((rc = upload(c, &L.cp.cl_own, gb.own))) return rc;
    if ((rc = upload(c, &L.cp.cl_nbr, gb.nbr))) return rc;
    // entry 0 is read (and not used) by lanes beyond a group's count, so a
    // level whose groups have no external node still gets one (a node index)
    if (gb.ext.empty()) gb.ext.push_back(0);
    if ((rc = upload(c, &L.cp.ext_src, gb.ext))) return rc;
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.cp.cl_coef, 9 * std::max<size_t>(1, gb.node.size())));
    if (mixed) MGFEM_HIP_TRY(ctx_alloc_t(c, &L.cp.cl_coef32, 9 * std::max<size_t>(1, gb.node.size())));
    if (!gb.node.empty())
      hipLaunchKernelGGL(k_gather_coef, dim3((unsigned)((gb.node.size() + 255) / 256)), dim3(256), 0, c->s, L.A,
                         L.n, L.cp.cl_node, (int)gb.node.size(), L.cp.cl_coef, L.cp.cl_coef32);
    MGFEM_HIP_TRY(hipGetLastError());
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  }

  // --- single-workgroup coarse part: as many coarsest levels as fit in LDS
  struct LevHost {
    int W, H, ox, oy, nstored, ncut, nact;
    std::vector<int16_t> slot, cutl, actl;
    std::vector<double> coef;
    int cut_off[5], act_off[5];
  };
  std::vector<LevHost> hosts;
  int total64 = 0;
  int lc = nl;
  for (int l = nl - 1; l >= 1 && nl - l <= 12; --l) {
    Level& L = c->lv[l];
    if (L.N > 256) break;
    LevHost h{};
    h.ox = L.bbox[0] - 1;
    h.oy = L.bbox[2] - 1;
    h.W = L.bbox[1] - L.bbox[0] + 3;
    h.H = L.bbox[3] - L.bbox[2] + 3;
    if (L.empty()) {
      h.ox = h.oy = 0;
      h.W = h.H = 3;
    }
    const int nb = h.W * h.H;
    if (nb > 32000) break;
    std::vector<uint8_t> fl(L.n);
    std::vector<double> A(9 * L.n);
    MGFEM_HIP_TRY(hipMemcpyAsync(fl.data(), L.flags, L.n, hipMemcpyDeviceToHost, c->s));
    MGFEM_HIP_TRY(hipMemcpyAsync(A.data(), L.A, 9 * L.n * sizeof(double), hipMemcpyDeviceToHost, c->s));
    std::vector<int> cl(std::max(1, L.cut_off[4]));
    if (L.cut_off[4] > 0)
      MGFEM_HIP_TRY(hipMemcpyAsync(cl.data(), L.cut_list, L.cut_off[4] * sizeof(int), hipMemcpyDeviceToHost, c->s));
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
    const bool coarsest = l == nl - 1;
    h.slot.assign(nb, -2);
    h.nstored = 0;
    std::vector<int16_t> bycol[4];
    const int pl[8] = {0, 1, 2, 3, 5, 6, 7, 8};
    for (int q = 0; q < nb; ++q) {
      const int gi = h.ox + q % h.W, gj = h.oy + q / h.W;
      if (gi < 0 || gj < 0 || gi > L.N || gj > L.N) continue;
      const int64_t k = gi + (int64_t)gj * L.stride;
      const uint8_t f = fl[k];
      if (!(f & kFlagActive)) continue;  // the outer ring of the box is never active
      if (coarsest) bycol[0].push_back((int16_t)q);  // ascending node order (the inverse's order)
      else bycol[(gi & 1) + 2 * (gj & 1)].push_back((int16_t)q);
      if (f & kFlagStored) {
        h.slot[q] = (int16_t)h.nstored++;
        for (int e = 0; e < 8; ++e) h.coef.push_back(A[pl[e] * L.n + k]);
        h.coef.push_back(A[4 * L.n + k]);
        h.coef.push_back(1.0 / A[4 * L.n + k]);
      } else {
        h.slot[q] = -1;
      }
    }
    if (h.nstored > 32000) break;
    h.act_off[0] = 0;
    for (int cc = 0; cc < 4; ++cc) {
      h.actl.insert(h.actl.end(), bycol[cc].begin(), bycol[cc].end());
      h.act_off[cc + 1] = (int)h.actl.size();
    }
    h.nact = (int)h.actl.size();
    h.ncut = coarsest ? 0 : L.cut_off[4];
    for (int cc = 0; cc < 5; ++cc) h.cut_off[cc] = coarsest ? 0 : L.cut_off[cc];
    for (int q = 0; q < h.ncut; ++q) {
      const int k = cl[q], gi = k % L.stride, gj = k / L.stride;
      h.cutl.push_back((int16_t)((gi - h.ox) + (gj - h.oy) * h.W));
    }
    auto bytes = [&](int ts) {
      int bsz = 3 * align16(nb * ts) + align16(h.nact * 2) + align16(nb * 2) + align16(10 * h.nstored * ts) +
                align16(h.ncut * 2);
      if (coarsest) bsz += align16(c->coarse_n * c->coarse_n * 8);
      return bsz;
    };
    if (coarsest && h.nact != c->coarse_n) {
      c->last_error = "coarsest active count mismatch";
      return MGFEM_ERR_HIP;
    }
    if (total64 + bytes(8) > (int)cap) break;
    total64 += bytes(8);
    hosts.insert(hosts.begin(), h);
    lc = l;
  }
  if (hosts.empty() || lc + (int)hosts.size() != nl) {
    c->last_error = "the coarsest grid does not fit in one workgroup's LDS";
    return MGFEM_ERR_UNSUPPORTED;
  }
  // descriptors: a float64 block and a float32 block (same layout, different LDS offsets)
  CoarsePlan& P = c->cplan;
  P.lc = lc;
  P.ndesc = (int)hosts.size();
  std::vector<int> desc;
  std::vector<double> coef;
  std::vector<int16_t> slot, cutl, actl;
  for (int pass = 0; pass < 2; ++pass) {
    const int ts = pass == 0 ? 8 : 4;
    // LDS: first the static block of every level (colour lists, row slots,
    // rows, cut lists, the coarsest inverse), padded to whole 1 KB chunks
    // (copied from the image), then the vectors x, b, r of every level
    // (zeroed in place)
    int off = 0, coef_off = 0, slot_off = 0, cut_off = 0, act_off = 0;
    std::vector<int> lev_desc(kDesc * P.ndesc, 0);
    for (int q = 0; q < P.ndesc; ++q) {
      const LevHost& h = hosts[q];
      const int nb = h.W * h.H;
      int* d = lev_desc.data() + kDesc * q;
      d[0] = c->lv[lc + q].N;
      d[1] = h.W;
      d[2] = h.H;
      d[3] = h.ox;
      d[4] = h.oy;
      d[5] = coef_off;
      d[6] = slot_off;
      for (int cc = 0; cc < 5; ++cc) d[7 + cc] = cut_off + h.cut_off[cc];
      d[15] = off;
      off += align16(h.nact * 2);
      d[16] = off;
      off += align16(nb * 2);
      d[17] = off;
      off += align16(10 * h.nstored * ts);
      d[18] = off;
      off += align16(h.ncut * 2);
      d[19] = h.nstored;
      if (q == P.ndesc - 1) {
        d[20] = off;
        off += align16(c->coarse_n * c->coarse_n * 8);
      }
      for (int cc = 0; cc < 5; ++cc) d[21 + cc] = act_off + h.act_off[cc];
      coef_off += h.nstored;
      slot_off += nb;
      cut_off += h.ncut;
      act_off += h.nact;
      if (pass == 0) {
        coef.insert(coef.end(), h.coef.begin(), h.coef.end());
        slot.insert(slot.end(), h.slot.begin(), h.slot.end());
        cutl.insert(cutl.end(), h.cutl.begin(), h.cutl.end());
        actl.insert(actl.end(), h.actl.begin(), h.actl.end());
      }
    }
    off = (off + 1023) / 1024 * 1024;
    if (pass == 0) P.static64 = off;
    else P.static32 = off;
    for (int q = 0; q < P.ndesc; ++q) {
      const LevHost& h = hosts[q];
      const int nb = h.W * h.H;
      int* d = lev_desc.data() + kDesc * q;
      d[12] = off;
      off += align16(nb * ts);
      d[13] = off;
      off += align16(nb * ts);
      d[14] = off;
      off += align16(nb * ts);
    }
    desc.insert(desc.end(), lev_desc.begin(), lev_desc.end());
    if (pass == 0) P.lds64 = off;
    else P.lds32 = off;
  }
  // LDS images: static parts at their offsets, vectors zero, the inverse
  // copied in on the device below
  std::vector<unsigned char> img[2];
  img[0].assign(P.static64, 0);
  img[1].assign(P.static32, 0);
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = 0; q < P.ndesc; ++q) {
      const LevHost& h = hosts[q];
      const int* d = desc.data() + kDesc * (pass * P.ndesc + q);
      unsigned char* b = img[pass].data();
      std::memcpy(b + d[15], h.actl.data(), h.actl.size() * 2);
      std::memcpy(b + d[16], h.slot.data(), h.slot.size() * 2);
      std::memcpy(b + d[18], h.cutl.data(), h.cutl.size() * 2);
      if (pass == 0) {
        std::memcpy(b + d[17], h.coef.data(), h.coef.size() * 8);
      } else {
        std::vector<float> f32(h.coef.begin(), h.coef.end());
        std::memcpy(b + d[17], f32.data(), f32.size() * 4);
      }
    }
  }
  int rc;
  if ((rc = upload(c, &P.img64, img[0]))) return rc;
  if ((rc = upload(c, &P.img32, img[1]))) return rc;
  {
    const int last64 = desc[kDesc * (P.ndesc - 1) + 20], last32 = desc[kDesc * (2 * P.ndesc - 1) + 20];
    const size_t ib = (size_t)c->coarse_n * c->coarse_n * sizeof(double);
    MGFEM_HIP_TRY(hipMemcpyAsync(P.img64 + last64, P.inv, ib, hipMemcpyDeviceToDevice, c->s));
    MGFEM_HIP_TRY(hipMemcpyAsync(P.img32 + last32, P.inv, ib, hipMemcpyDeviceToDevice, c->s));
  }
  if ((rc = upload(c, &P.desc, desc))) return rc;
  if ((rc = upload(c, &P.coef, coef))) return rc;
  if (mixed) {
    std::vector<float> c32(coef.begin(), coef.end());
    if ((rc = upload(c, &P.coef32, c32))) return rc;
  }
  if ((rc = upload(c, &P.slot, slot))) return rc;
  if ((rc = upload(c, &P.cutl, cutl))) return rc;
  if ((rc = upload(c, &P.actl, actl))) return rc;
  {
    // grid indices of the first coarse level's active nodes in its list order
    // (rows and columns of the coarse map)
    const LevHost& h = hosts[0];
    const int s0 = c->lv[lc].stride;
    std::vector<int> gidx(std::max(1, h.nact));
    for (int q = 0; q < h.nact; ++q)
      gidx[q] = (h.ox + h.actl[q] % h.W) + (h.oy + h.actl[q] / h.W) * s0;
    if ((rc = upload(c, &P.map.idx, gidx))) return rc;
    P.map.n = h.nact;
  }
  MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  set_kernel_attributes();
  return build_tile_lists(c);
}

}  // namespace mgfem
