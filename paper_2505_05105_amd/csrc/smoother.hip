// The multigrid cycle on the device (sections 3 and 5 of the paper).
//
// Smoothing step = one Gauss-Seidel sweep over the four colours
// c(i,j) = (i mod 2) + 2 (j mod 2), then eta sweeps restricted to the
// vertices of cut cells (the extra smoothing of section 5.3).  The 9-point
// stencil never couples two nodes of one colour, so a colour phase is a set of
// independent updates x_i += (b_i - (A x)_i) / a_ii.
//
// Kernels:
//  k_sweep      one full four-colour sweep of a TW x TH tile per workgroup.
//               The tile and a halo of 4 are staged in LDS; phase p updates
//               its colour on the tile grown by 3 - p, so the core is exact
//               without any exchange between workgroups.  Reads x from one
//               buffer and writes the core to the other (ping-pong), so halos
//               are never read while another workgroup writes them.  Tiles
//               are numbered so that consecutive tiles land on one XCD
//               (workgroups are dealt to the 8 XCDs round robin), which keeps
//               shared halos in that XCD's L2.
//  k_cut        all 4 eta phases of the extra smoothing of one group of cut
//               vertices in LDS (the group carries its dependency closure).
//               Cut-vertex values are read from the snapshot the preceding
//               kernel wrote, so no workgroup reads a value another one
//               is writing.
//  k_resrestrict  residual r = b - A x on a fine tile and its restriction
//               b_c = R r (weights 1, 1/2, 1/4) in one pass; zeroes x_c.
//  k_prolong    x += P x_c (bilinear) at active fine nodes.
//  k_coarse_apply  the coarse part of the cycle (from the first level with at
//               most a few thousand unknowns down) as one dense matrix-vector
//               product; the matrix is computed at set-up.
//  k_coarse     the cycle of the coarsest levels in one workgroup, the levels
//               in LDS: builds the dense map at set-up (one unit right-hand
//               side per workgroup) and runs where no map is kept.
//  k_*_multi    the same tile, group and row bodies for many problems in one
//               launch (batched solves): a table of per-problem arguments and
//               a list of (problem, unit) work items.
//  k_batched    the persistent alternative for batched solves: one workgroup
//               per problem, drawn from an atomic queue.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "mgfem_internal.h"

namespace mgfem {
namespace {

constexpr int kHalo = 4;
// threads of a cut-group workgroup (a compile-time block size: reading blockDim
// costs a load from the dispatch packet)
constexpr int kCutThreads = 256;
// threads of the single-workgroup coarse cycle: the levels it runs hold at
// most a few thousand nodes, so few waves keep its many barriers cheap
constexpr int kCoarseThreads = 256;

template <class T>
struct SweepArgs {
  const T* xin;
  T* xout;
  const T* b;
  const T* A;
  const uint8_t* fl;
  const int* cutpos;
  T* snap;
  int N, s;
  int64_t n;
  int i0, j0, i1, j1;  // bounding box of active nodes
  int ntx, nty, per;   // tiles and tiles per XCD
  const int* tiles;    // active tiles (row-major tile indices), or null for all
  int ntiles;
  int reverse;
  // optional residual norm of the incoming iterate (float64 only): per-tile
  // partials, a completion counter and the final (max |r|, sum r^2)
  double* part;
  int norm;
  const T* xc;  // coarse iterate to prolongate into the staged tile, or null
  int sc;
  // tile plan (see Level): stored rows and core cut vertices of each tile
  const int* tmeta;
  const int* tp_off;
  const int* tp_idx;
  const T* tp_coef;
  const int* tc_off;
  const int* tc_idx;
  const int* tc_pos;
  const T* zero;  // at least 16 zero bytes: the source of staged groups off the grid
};

__device__ inline double nanmax2(double a, double b) { return (b > a || b != b) ? b : a; }

// product of the stored stencil row at node k with LDS values around q
template <class T, int RW>
__device__ inline T stored_offdiag(const T* __restrict__ A, int64_t n, int64_t k, const T* su, int q) {
  T acc = A[k] * su[q - RW - 1];
  acc += A[n + k] * su[q - RW];
  acc += A[2 * n + k] * su[q - RW + 1];
  acc += A[3 * n + k] * su[q - 1];
  acc += A[5 * n + k] * su[q + 1];
  acc += A[6 * n + k] * su[q + RW - 1];
  acc += A[7 * n + k] * su[q + RW];
  acc += A[8 * n + k] * su[q + RW + 1];
  return acc;
}

// the same off-diagonal product from a row kept in LDS (cf: 9 coefficients)
template <class T, int RW>
__device__ inline T lds_offdiag(const T* cf, const T* su, int q) {
  T acc = cf[0] * su[q - RW - 1];
  acc += cf[1] * su[q - RW];
  acc += cf[2] * su[q - RW + 1];
  acc += cf[3] * su[q - 1];
  acc += cf[5] * su[q + 1];
  acc += cf[6] * su[q + RW - 1];
  acc += cf[7] * su[q + RW];
  acc += cf[8] * su[q + RW + 1];
  return acc;
}

template <class T, int RW>
__device__ inline T q1_neighbours(const T* su, int q) {
  return (su[q - RW - 1] + su[q - RW] + su[q - RW + 1]) + (su[q - 1] + su[q + 1]) +
         (su[q + RW - 1] + su[q + RW] + su[q + RW + 1]);
}

// Gauss-Seidel value of one node: x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii.
// Interior Q1 rows (centre 8/3, neighbours -1/3) give (3 b_i + sum x_j) / 8.
template <class T, int RW>
__device__ inline T gs_value(const T* __restrict__ A, int64_t n, int64_t k, bool stored, const T* su, int q,
                             T bv) {
  if (stored) return (bv - stored_offdiag<T, RW>(A, n, k, su, q)) / A[4 * n + k];
  return (T(3) * bv + q1_neighbours<T, RW>(su, q)) * T(0.125);
}

// One full four-colour sweep of a TW x TH tile.  The iterate is staged in
// LDS (tile plus a halo of 4) together with the tile plan's stored rows; each
// thread prefetches the flags and right-hand sides of the nodes it updates in
// the four phases into registers.  A node's value is final after the phase of
// its colour, so core nodes are written out right there.
//  prolong: the staged iterate is x + P x_c (the coarse-grid correction is
//           applied on the fly, so the first post-smoothing sweep needs no
//           separate prolongation pass).
//  norm:    before the first phase, the residual of the incoming iterate on
//           the core is reduced into per-tile partials (max |r|, sum r^2).
// final reduction of (max, sum) pairs in a fixed order: each of the 1024
// threads takes the pairs in chunks of four, the loads of a chunk issued
// together (a lane beyond nb reads pair 0 and drops it: loads under a branch
// would wait for one another), then a wave reduction and the 16 waves in
// order
__global__ __launch_bounds__(1024) void k_reduce_pairs(const double* __restrict__ part, int nb, double* __restrict__ out, double* host_out,
                               double* seq) {
  __shared__ double smx[16], ssm[16];
  constexpr int U = 4;
  double mx = 0.0, sm = 0.0;
  for (int base = 0; base < nb; base += U * 1024) {
    double lm[U], ls[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = base + threadIdx.x + u * 1024;
      const int qq = q < nb ? q : 0;
      lm[u] = part[2 * qq];
      ls[u] = part[2 * qq + 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = base + (int)threadIdx.x + u * 1024 < nb;
      mx = nanmax2(mx, in ? lm[u] : 0.0);
      sm += in ? ls[u] : 0.0;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mx = nanmax2(mx, __shfl_xor(mx, o));
    sm += __shfl_xor(sm, o);
  }
  if ((threadIdx.x & 63) == 0) {
    smx[threadIdx.x >> 6] = mx;
    ssm[threadIdx.x >> 6] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) {
      mx = nanmax2(mx, smx[w]);
      sm += ssm[w];
    }
    out[0] = mx;
    out[1] = sm;
    const double q = seq[0] + 1.0;  // counted on the device (graph replays)
    seq[0] = q;
    double* rec = host_out + 4 * (int)((long long)q % kRedSlots);
    rec[0] = mx;  // straight to pinned host memory; the sequence number goes last
    rec[1] = sm;
    __threadfence_system();
    rec[2] = q;
    __threadfence_system();
  }
}

// 16 bytes per lane from global memory straight into LDS at dst + 16 * lane
// (a device function: the builtin's 16-byte form exists only for gfx950)
__device__ inline void lds_load16(const void* src, void* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// the sweep of tile t of the level's tile list (one workgroup)
template <class T, int TW, int TH, int BS>
__device__ void sweep_tile(const SweepArgs<T>& a, const int t) {
  constexpr int RW = TW + 2 * kHalo, RH = TH + 2 * kHalo;
  constexpr int NU = (RW * RH + BS - 1) / BS;
  constexpr int NXM = (RW - 1) / 2, NYM = (RH - 1) / 2;  // colour nodes per row/column, phase 0 bound
  constexpr int NP = (NXM * NYM + BS - 1) / BS;          // phase nodes per thread
  constexpr int PR = 255;  // stored rows of a tile kept in LDS (slot 255: read A)
  constexpr int NCF = (9 * PR + BS - 1) / BS, NRI = (PR + BS - 1) / BS;
  constexpr int KC = 2;                             // core cut vertices prefetched per thread
  constexpr int G = 16 / (int)sizeof(T);  // values per 16-byte lane load: G consecutive nodes of a row
  static_assert(RW % G == 0, "region rows hold whole 16-byte groups");
  constexpr int NQ = RW * RH / G, NCH = (NQ + 63) / 64;
  __shared__ __align__(16) T su[NCH * 64 * G];  // the region, rounded up to whole 64-group chunks
  // coarse tile under the region (fused prolongation): parents of the region's
  // nodes, rows padded to whole groups
  constexpr int CW = (RW / 2 + 2 + G - 1) / G * G, CH = RH / 2 + 2;
  constexpr int NCQ = CW * CH / G, NCCH = (NCQ + 63) / 64;
  __shared__ __align__(16) T sxc[NCCH * 64 * G];
  __shared__ T scf[9 * PR];
  __shared__ uint8_t sslot[RH * RW];  // stored node: its row in scf (255: read A); others unused
  // tile, plan offsets and counts in one uniform 32-byte load
  const int* mt = a.tmeta + 8 * t;
  const int tile = mt[0], p0 = mt[1], nrow = mt[2], c0 = mt[3], ncut = mt[4];
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const int ox = a.i0 + tx * TW - kHalo, oy = a.j0 + ty * TH - kHalo;
  const int tid = threadIdx.x;
  // this thread's nodes in each phase (LDS index, or -1), with flags and b
  int pq[4][NP];
  uint8_t pf[4][NP];
  T pb[4][NP];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int c = a.reverse ? 3 - p : p;
    const int lo = p + 1, hix = RW - 1 - p, hiy = RH - 1 - p;
    const int fx = lo + (((c & 1) - (ox + lo)) & 1), fy = lo + (((c >> 1) - (oy + lo)) & 1);
    const int nxm = (hix - lo + 1) / 2, nym = (hiy - lo + 1) / 2;
#pragma unroll
    for (int it = 0; it < NP; ++it) {
      const int q = tid + BS * it;
      const int ri = fx + 2 * (q % nxm), rj = fy + 2 * (q / nxm);
      const int gi = ox + ri, gj = oy + rj;
      const bool ok = q < nxm * nym && ri < hix && rj < hiy && gi >= 0 && gj >= 0 && gi <= a.N && gj <= a.N;
      pq[p][it] = ok ? ri + rj * RW : -1;
      pf[p][it] = ok ? a.fl[gi + (int64_t)gj * a.s] : 0;
    }
  }
  // the tile plan: rows of its stored nodes, its core cut vertices
  const int nrl = min(nrow, PR);
  T rcf[NCF];
  int rix[NRI];
#pragma unroll
  for (int u = 0; u < NCF; ++u) {
    const int q = tid + u * BS;
    rcf[u] = q < 9 * nrl ? a.tp_coef[9 * (int64_t)p0 + q] : T(0);
  }
#pragma unroll
  for (int u = 0; u < NRI; ++u) {
    const int e = tid + u * BS;
    rix[u] = e < nrl ? a.tp_idx[p0 + e] : -1;
  }
  // the staged iterate goes straight from global memory into LDS: 16 bytes
  // (one group) per lane, 64 groups per wave instruction, no registers. A
  // group that lies only partly on the grid loads zeros here; its on-grid
  // nodes are filled in after the loads have landed.
  const int lane = tid & 63, wave = tid >> 6;
  for (int ch = wave; ch < NCH; ch += BS / 64) {
    const int e = (ch * 64 + lane) * G;
    const int gi = ox + e % RW, gj = oy + e / RW;
    const bool in = e < RW * RH && gi >= 0 && gj >= 0 && gi + G - 1 <= a.N && gj <= a.N;
    lds_load16(in ? a.xin + gi + (int64_t)gj * a.s : a.zero, su + ch * 64 * G);
  }
  // the coarse iterate under the region, the same way (fused prolongation)
  const int cox = ox >> 1, coy = oy >> 1;  // floor: the parents of the region's first node
  const int Nc = a.N >> 1;
  if (a.xc) {
    for (int ch = wave; ch < NCCH; ch += BS / 64) {
      const int e = (ch * 64 + lane) * G;
      const int I = cox + e % CW, J = coy + e / CW;
      const bool in = e < CW * CH && I >= 0 && J >= 0 && I + G - 1 <= Nc && J <= Nc;
      lds_load16(in ? a.xc + I + (int64_t)J * a.sc : a.zero, sxc + ch * 64 * G);
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int it = 0; it < NP; ++it) {
      const int q = pq[p][it];
      pb[p][it] = q >= 0 ? a.b[(ox + q % RW) + (int64_t)(oy + q / RW) * a.s] : T(0);
    }
  // the core's cut vertices (used after the last phase), issued last so that
  // waiting for them never holds back the loads above
  int cix[KC], cpo[KC];
#pragma unroll
  for (int u = 0; u < KC; ++u) {
    const int e = tid + u * BS;
    cix[u] = e < ncut ? a.tc_idx[c0 + e] : -1;
    cpo[u] = e < ncut ? a.tc_pos[c0 + e] : 0;
  }
#pragma unroll
  for (int u = 0; u < NCF; ++u) {
    const int q = tid + u * BS;
    if (q < 9 * nrl) scf[q] = rcf[u];
  }
#pragma unroll
  for (int u = 0; u < NRI; ++u)
    if (rix[u] >= 0) sslot[rix[u]] = (uint8_t)(tid + u * BS);
  for (int e = PR + tid; e < nrow; e += BS) sslot[a.tp_idx[p0 + e]] = (uint8_t)PR;  // beyond the LDS rows
  __builtin_amdgcn_s_waitcnt(0);  // the global->LDS loads of this thread have landed
  __syncthreads();
  if (ox < 0 || ox + RW > a.N + 1 || (a.xc && (cox < 0 || cox + CW > Nc + 1))) {
    // the tile meets a side of the grid: on-grid nodes of straddling groups
    for (int ch = wave; ch < NCH; ch += BS / 64) {
      const int e = (ch * 64 + lane) * G;
      const int gi = ox + e % RW, gj = oy + e / RW;
      if (e < RW * RH && gj >= 0 && gj <= a.N && (gi < 0 || gi + G - 1 > a.N))
        for (int v = 0; v < G; ++v)
          if (gi + v >= 0 && gi + v <= a.N) su[e + v] = a.xin[gi + v + (int64_t)gj * a.s];
    }
    if (a.xc)
      for (int ch = wave; ch < NCCH; ch += BS / 64) {
        const int e = (ch * 64 + lane) * G;
        const int I = cox + e % CW, J = coy + e / CW;
        if (e < CW * CH && J >= 0 && J <= Nc && (I < 0 || I + G - 1 > Nc))
          for (int v = 0; v < G; ++v)
            if (I + v >= 0 && I + v <= Nc) sxc[e + v] = a.xc[I + v + (int64_t)J * a.sc];
      }
    __syncthreads();
  }
  if (a.xc) {
    // + P x_c: bilinear interpolation from the (up to) four coarse parents,
    // written without branches (for an even index both parents coincide)
#pragma unroll
    for (int it = 0; it < NU; ++it) {
      const int q = tid + BS * it;
      const int gi = ox + q % RW, gj = oy + q / RW;
      if (q < RW * RH && gi >= 0 && gj >= 0 && gi <= a.N && gj <= a.N) {
        const int I0 = (gi >> 1) - cox, I1 = ((gi + 1) >> 1) - cox;
        const int J0 = ((gj >> 1) - coy) * CW, J1 = (((gj + 1) >> 1) - coy) * CW;
        su[q] += T(0.25) * ((sxc[I0 + J0] + sxc[I1 + J0]) + (sxc[I0 + J1] + sxc[I1 + J1]));
      }
    }
    __syncthreads();
  }
  auto in_core = [&](int q) {
    const int ri = q % RW, rj = q / RW;
    return ri >= kHalo && ri < kHalo + TW && rj >= kHalo && rj < kHalo + TH && ox + ri <= a.i1 && oy + rj <= a.j1;
  };
  if (a.norm) {
    __shared__ double smx[BS / 64], ssm[BS / 64];
    double mx = 0.0, sm = 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int it = 0; it < NP; ++it) {
        const int q = pq[p][it];
        if (q < 0 || !(pf[p][it] & kFlagActive) || !in_core(q)) continue;
        T ax;
        if (pf[p][it] & kFlagStored) {
          const int sl = sslot[q];
          if (sl < PR) {
            ax = scf[9 * sl + 4] * su[q] + lds_offdiag<T, RW>(scf + 9 * sl, su, q);
          } else {
            const int64_t k = (ox + q % RW) + (int64_t)(oy + q / RW) * a.s;
            ax = a.A[4 * a.n + k] * su[q] + stored_offdiag<T, RW>(a.A, a.n, k, su, q);
          }
        } else {
          ax = T(8) / T(3) * su[q] - q1_neighbours<T, RW>(su, q) * T(1.0 / 3.0);
        }
        const double r = (double)(pb[p][it] - ax);
        mx = nanmax2(mx, fabs(r));
        sm += r * r;
      }
    for (int o = 32; o > 0; o >>= 1) {
      mx = nanmax2(mx, __shfl_xor(mx, o));
      sm += __shfl_xor(sm, o);
    }
    if ((tid & 63) == 0) {
      smx[tid >> 6] = mx;
      ssm[tid >> 6] = sm;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < BS / 64; ++w) {
        mx = nanmax2(mx, smx[w]);
        sm += ssm[w];
      }
      a.part[2 * t] = mx;
      a.part[2 * t + 1] = sm;
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
#pragma unroll
    for (int it = 0; it < NP; ++it) {
      const int q = pq[p][it];
      const uint8_t f = pf[p][it];
      if (q < 0 || !(f & kFlagActive)) continue;
      const int64_t k = (ox + q % RW) + (int64_t)(oy + q / RW) * a.s;
      T v;
      if (f & kFlagStored) {
        const int sl = sslot[q];
        v = sl < PR ? (pb[p][it] - lds_offdiag<T, RW>(scf + 9 * sl, su, q)) / scf[9 * sl + 4]
                    : gs_value<T, RW>(a.A, a.n, k, true, su, q, pb[p][it]);
      } else {
        v = gs_value<T, RW>(a.A, a.n, k, false, su, q, pb[p][it]);
      }
      su[q] = v;
      if (in_core(q)) a.xout[k] = v;
    }
    __syncthreads();
  }
  // snapshot of the core's cut vertices (final after their colour's phase)
#pragma unroll
  for (int u = 0; u < KC; ++u)
    if (cix[u] >= 0) a.snap[cpo[u]] = su[cix[u]];
  for (int e = tid + KC * BS; e < ncut; e += BS) a.snap[a.tc_pos[c0 + e]] = su[a.tc_idx[c0 + e]];
}

// Work lists of a launch are dealt to the eight XCDs in contiguous eighths
// (workgroups are dealt to the XCDs round robin), so that neighbouring tiles
// of one level share an XCD's L2.
__device__ inline int xcd_item(int per) { return (blockIdx.x & 7) * per + (blockIdx.x >> 3); }

// The float 64 x 16 instance is held to 64 registers, so that four of its
// workgroups share a CU and the N = 2048 level's tiles start in one round
// (the float64 instance would spill at that bound).
template <class T, int TW, int TH, int BS>
__global__ __launch_bounds__(BS, (sizeof(T) == 4 && TW == 64 && TH == 16) ? 8 : 1) void k_sweep(SweepArgs<T> a) {
  const int t = xcd_item(a.per);
  if (t >= a.ntiles) return;  // uniform for the whole block, before any barrier
  sweep_tile<T, TW, TH, BS>(a, t);
}

// Several problems in one launch (batched solves): one entry per problem
// with the arguments of its level and both ping-pong buffers of the level
// and of the next coarser one; the work list holds (problem, tile) pairs.
// par is the level's parity (which buffer holds the iterate), parc that of
// the coarser level, except for problems whose coarser level is the first
// level of their coarse part (its iterate is always buffer 0).
template <class T>
struct SweepEntry {
  SweepArgs<T> a;
  T* X[2];
  const T* XC[2];
  int xc_fixed;
};

template <class T, int TW, int TH, int BS>
__global__ __launch_bounds__(BS) void k_sweep_multi(const SweepEntry<T>* tab, const int2* work, int nwork,
                                                    int par, int parc, int prolong) {
  const int i = xcd_item((nwork + 7) >> 3);
  if (i >= nwork) return;
  const int2 w = work[i];
  const SweepEntry<T>& E = tab[w.x];
  SweepArgs<T> a = E.a;
  a.xin = E.X[par];
  a.xout = E.X[1 - par];
  a.xc = prolong ? E.XC[E.xc_fixed ? 0 : parc] : nullptr;
  sweep_tile<T, TW, TH, BS>(a, w.y);
}

// extra smoothing of one group of cut vertices, all phases in LDS
template <class T>
struct CutArgs {
  const int* g_info;
  const int* cl_node;
  const int* cl_q;
  const uint8_t* cl_own;
  const int16_t* cl_nbr;
  const int* ext_src;
  const T* cl_coef;  // per closure node: 8 off-diagonals (planes 0,1,2,3,5,6,7,8) and 1/diagonal
  T* x;
  const T* b;
  const T* snap;
  int eta, reverse;
};


struct alignas(16) Refs8 {
  int16_t r[8];
};

// the eta sweeps of cut group g (one workgroup of 256 threads; smem: the
// group's dynamic LDS)
template <class T>
__device__ void cut_group(const CutArgs<T>& a, const int g, unsigned char* smem) {
  const int* gi = a.g_info + 9 * g;
  const int cl_off = gi[0], cl_cnt = gi[1], ext_off = gi[2], ext_cnt = gi[3];
  // the colour ranges in registers: a value read from global memory after a
  // workgroup barrier is loaded again (the barrier orders global memory too),
  // and that load would sit in every colour phase
  int cr[5];
#pragma unroll
  for (int e = 0; e < 5; ++e) cr[e] = gi[4 + e];
  const CutLds lay = cut_lds_layout(cl_cnt, ext_cnt, (int)sizeof(T));
  T* vals = reinterpret_cast<T*>(smem + lay.vals);
  T* sb = reinterpret_cast<T*>(smem + lay.b);
  T* sinv = reinterpret_cast<T*>(smem + lay.invd);
  T* scoef = reinterpret_cast<T*>(smem + lay.coef);
  Refs8* srefs = reinterpret_cast<Refs8*>(smem + lay.refs);
  const Refs8* grefs = reinterpret_cast<const Refs8*>(a.cl_nbr) + cl_off;
  auto stage = [&](int t) {
    const int64_t k = a.cl_node[cl_off + t];
    const T v = a.snap[a.cl_q[cl_off + t]];
    const T bv = a.b[k];
    const T* cg = a.cl_coef + 9 * (int64_t)(cl_off + t);
    T cf[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) cf[e] = cg[e];
    const Refs8 rr = grefs[t];
    vals[t] = v;
    sb[t] = bv;
    sinv[t] = cf[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) scoef[e * cl_cnt + t] = cf[e];
    srefs[t] = rr;
    return k;
  };
  // The first closure node and the first external node of this thread are
  // staged in two rounds of global loads: every index and row load, then
  // every value load they point at, then the LDS stores.  The stores do not
  // branch (a lane beyond the counts loads entry 0 of the arrays, which a
  // level with groups always has, and stores into its own slot of the dump
  // area), since a store under a branch lets the compiler move the loads
  // that feed it under the branch too, one node after the other.  The second
  // closure node of each thread (groups of more than 256 nodes, a uniform
  // test) and nodes beyond take the same path and the loops after.  The
  // first KW nodes keep their grid index and ownership in registers for the
  // write-back at the end.  Coefficients lie in LDS plane by plane
  // (coefficient e of node t at e * cl_cnt + t), so that consecutive lanes
  // store and load consecutive words.
  constexpr int KW = 2;
  int64_t wk[KW] = {0, 0};
  uint8_t wo[KW] = {0, 0};
  const int lane = threadIdx.x & 63;
  T* dump = reinterpret_cast<T*>(smem + lay.dump);
  auto stage2 = [&](int u, bool with_ext) {
    const int t = threadIdx.x + u * kCutThreads;
    const bool in = t < cl_cnt;
    const int e = in ? cl_off + t : 0;
    const int64_t k = a.cl_node[e];
    const int q = a.cl_q[e];
    const uint8_t own = a.cl_own[e];
    const T* cg = a.cl_coef + 9 * (int64_t)e;
    T cf[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) cf[c] = cg[c];
    const Refs8 rr = reinterpret_cast<const Refs8*>(a.cl_nbr)[e];
    const int te = threadIdx.x;
    const int src = with_ext ? a.ext_src[te < ext_cnt ? ext_off + te : 0] : 0;
    const T v = a.snap[q];
    const T bv = a.b[k];
    const T ev = with_ext ? *(src >= 0 ? a.x + src : a.snap + (-(1 + src))) : T(0);
    *(in ? vals + t : dump + lane) = v;
    *(in ? sb + t : dump + lane) = bv;
    *(in ? sinv + t : dump + lane) = cf[8];
    T* pc = in ? scoef + t : dump + lane;
    const int cs = in ? cl_cnt : 64;
#pragma unroll
    for (int c = 0; c < 8; ++c) pc[c * cs] = cf[c];
    *(in ? srefs + t : reinterpret_cast<Refs8*>(dump) + lane) = rr;
    if (with_ext) *(te <= ext_cnt ? vals + cl_cnt + te : dump + lane) = te < ext_cnt ? ev : T(0);
    wk[u] = k;
    wo[u] = in ? own : 0;
  };
  stage2(0, true);
  if (cl_cnt > kCutThreads) stage2(1, false);
  for (int t = threadIdx.x + KW * kCutThreads; t < cl_cnt; t += kCutThreads) stage(t);
  for (int t = threadIdx.x + kCutThreads; t <= ext_cnt; t += kCutThreads) {
    T v = T(0);
    if (t < ext_cnt) {
      const int src = a.ext_src[ext_off + t];
      v = src >= 0 ? a.x[src] : a.snap[-(1 + src)];
    }
    vals[cl_cnt + t] = v;
  }
  __syncthreads();
  // this thread's first node of every colour, with its row, kept in registers
  // across the 4 eta phases (a phase then only reads neighbour values)
  int rt[4];
  Refs8 rrf[4];
  T rb[4], rinv[4], rcf[4][8];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int t = cr[c] + threadIdx.x;
    rt[c] = t < cr[c + 1] ? t : -1;
    const int tt = rt[c] >= 0 ? t : 0;
    rrf[c] = srefs[tt];
    rb[c] = sb[tt];
    rinv[c] = sinv[tt];
#pragma unroll
    for (int e = 0; e < 8; ++e) rcf[c][e] = scoef[e * cl_cnt + tt];
  }
  // one colour phase; called with a literal colour so that the register
  // arrays above are indexed by constants (a run-time index would move them
  // to scratch memory)
  auto phase = [&](const int c) {
    if (rt[c] >= 0) {
      T nb[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) nb[e] = vals[rrf[c].r[e]];
      T acc = rb[c];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc -= rcf[c][e] * nb[e];
      vals[rt[c]] = acc * rinv[c];
    }
    const int lo = cr[c] + kCutThreads, hi = cr[c + 1];
    for (int t = lo + threadIdx.x; t < hi; t += kCutThreads) {
      const Refs8 rr = srefs[t];
      T nb[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) nb[e] = vals[rr.r[e]];
      T acc = sb[t];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc -= scoef[e * cl_cnt + t] * nb[e];
      vals[t] = acc * sinv[t];
    }
    __syncthreads();
  };
  if (!a.reverse) {
    for (int sweep = 0; sweep < a.eta; ++sweep) {
      phase(0);
      phase(1);
      phase(2);
      phase(3);
    }
  } else {
    for (int sweep = 0; sweep < a.eta; ++sweep) {
      phase(3);
      phase(2);
      phase(1);
      phase(0);
    }
  }
#pragma unroll
  for (int u = 0; u < KW; ++u)
    if (wo[u]) a.x[wk[u]] = vals[threadIdx.x + u * kCutThreads];
  for (int t = threadIdx.x + KW * kCutThreads; t < cl_cnt; t += kCutThreads)
    if (a.cl_own[cl_off + t]) a.x[a.cl_node[cl_off + t]] = vals[t];
}

template <class T>
__global__ __launch_bounds__(kCutThreads) void k_cut(CutArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  cut_group<T>(a, blockIdx.x, smem);
}

template <class T>
struct CutEntry {
  CutArgs<T> a;
  T* X[2];
};

template <class T>
__global__ __launch_bounds__(kCutThreads) void k_cut_multi(const CutEntry<T>* tab, const int2* work, int nwork, int par) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int i = xcd_item((nwork + 7) >> 3);
  if (i >= nwork) return;
  const int2 w = work[i];
  const CutEntry<T>& E = tab[w.x];
  CutArgs<T> a = E.a;
  a.x = E.X[par];
  cut_group<T>(a, w.y, smem);
}

// one colour phase over a list of nodes (used when a level has no group plan)
template <class T>
__global__ void k_gs_list(const T* __restrict__ A, const uint8_t* __restrict__ fl, T* x, const T* __restrict__ b,
                          int N, int64_t n, const int* __restrict__ list, int cnt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const int s = N + 1;
  const int64_t k = list[t];
  const int i = (int)(k % s), j = (int)(k / s);
  T diag = A[4 * n + k];
  T acc = b[k] - diag * x[k];
  for (int p = 0; p < 9; ++p) {
    if (p == 4) continue;
    const int ii = i + p % 3 - 1, jj = j + p / 3 - 1;
    if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
    acc -= A[p * n + k] * x[ii + (int64_t)jj * s];
  }
  x[k] += acc / diag;
  (void)fl;
}

template <class T>
struct ResArgs {
  const T* x;
  const T* b;
  const T* A;
  const uint8_t* fl;
  int N, s;
  int64_t n;
  T* bc;
  T* xc;
  const uint8_t* flc;
  const int* cutposc;
  T* snapc;
  int Nc, sc;
  int I0, J0, I1, J1;  // coarse bounding box
  int ntx, nty, per;
  const int* tiles;  // coarse tiles that hold an active coarse node
  int ntiles;
};

template <class T, int RW>
__device__ inline T row_product(const T* __restrict__ A, int64_t n, int64_t k, bool stored, const T* su, int q) {
  if (stored) return A[4 * n + k] * su[q] + stored_offdiag<T, RW>(A, n, k, su, q);
  return T(8) / T(3) * su[q] - q1_neighbours<T, RW>(su, q) * T(1.0 / 3.0);
}

// residual and restriction of coarse tile t of the level's list
template <class T, int CW, int CH, int BS>
__device__ void rr_tile(const ResArgs<T>& a, const int t) {
  constexpr int RW = 2 * CW + 1, RH = 2 * CH + 1;  // fine residual region
  constexpr int UW = RW + 2, UH = RH + 2;          // fine x region
  constexpr int NU = (UW * UH + BS - 1) / BS, NR = (RW * RH + BS - 1) / BS;
  __shared__ T su[UH * UW];
  __shared__ T sr[RH * RW];
  const int tile = a.tiles[t];
  const int tid = threadIdx.x;
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const int cI0 = a.I0 + tx * CW, cJ0 = a.J0 + ty * CH;
  const int fx0 = 2 * cI0 - 1, fy0 = 2 * cJ0 - 1;  // residual region origin
  const int ux0 = fx0 - 1, uy0 = fy0 - 1;
  uint8_t rf[NR];
  T rb[NR];
  {
    T ru[NU];
#pragma unroll
    for (int it = 0; it < NU; ++it) {
      const int q = tid + BS * it;
      const int gi = ux0 + q % UW, gj = uy0 + q / UW;
      ru[it] = (q < UW * UH && gi >= 0 && gj >= 0 && gi <= a.N && gj <= a.N) ? a.x[gi + (int64_t)gj * a.s] : T(0);
    }
    // flags and b together (b of an inactive node is loaded and never used),
    // so that no load waits for another
#pragma unroll
    for (int it = 0; it < NR; ++it) {
      const int q = tid + BS * it;
      const int gi = fx0 + q % RW, gj = fy0 + q / RW;
      const bool in = q < RW * RH && gi >= 0 && gj >= 0 && gi <= a.N && gj <= a.N;
      rf[it] = in ? a.fl[gi + (int64_t)gj * a.s] : 0;
      rb[it] = in ? a.b[gi + (int64_t)gj * a.s] : T(0);
    }
#pragma unroll
    for (int it = 0; it < NU; ++it) {
      const int q = tid + BS * it;
      if (q < UW * UH) su[q] = ru[it];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NR; ++it) {
    const int q = tid + BS * it;
    if (q >= RW * RH) break;
    const int ri = q % RW, rj = q / RW;
    T r = T(0);
    if (rf[it] & kFlagActive) {
      const int64_t k = (fx0 + ri) + (int64_t)(fy0 + rj) * a.s;
      r = rb[it] - row_product<T, UW>(a.A, a.n, k, (rf[it] & kFlagStored) != 0, su, (ri + 1) + (rj + 1) * UW);
    }
    sr[q] = r;
  }
  __syncthreads();
  for (int q = tid; q < CW * CH; q += BS) {
    const int I = cI0 + q % CW, J = cJ0 + q / CW;
    if (I > a.I1 || J > a.J1) continue;
    const int64_t kc = I + (int64_t)J * a.sc;
    const uint8_t f = a.flc[kc];
    if (!(f & kFlagActive)) continue;
    const int ci = 2 * (q % CW) + 1, cj = 2 * (q / CW) + 1;  // centre in the residual region
    const T* r0 = sr + ci + cj * RW;
    const T mid = r0[0] + T(0.5) * (r0[-1] + r0[1]);
    const T lo = r0[-RW] + T(0.5) * (r0[-RW - 1] + r0[-RW + 1]);
    const T hi = r0[RW] + T(0.5) * (r0[RW - 1] + r0[RW + 1]);
    a.bc[kc] = mid + T(0.5) * (lo + hi);
    a.xc[kc] = T(0);
    if (f & kFlagCut) a.snapc[a.cutposc[kc]] = T(0);
  }
}

template <class T, int CW, int CH, int BS>
__global__ __launch_bounds__(BS) void k_resrestrict(ResArgs<T> a) {
  const int t = xcd_item(a.per);
  if (t >= a.ntiles) return;  // uniform for the whole block, before any barrier
  rr_tile<T, CW, CH, BS>(a, t);
}

template <class T>
struct RrEntry {
  ResArgs<T> a;
  const T* X[2];
  T* XC[2];
  int xc_fixed;
};

template <class T, int CW, int CH, int BS>
__global__ __launch_bounds__(BS) void k_resrestrict_multi(const RrEntry<T>* tab, const int2* work, int nwork,
                                                          int par, int parc) {
  const int i = xcd_item((nwork + 7) >> 3);
  if (i >= nwork) return;
  const int2 w = work[i];
  const RrEntry<T>& E = tab[w.x];
  ResArgs<T> a = E.a;
  a.x = E.X[par];
  a.xc = E.XC[E.xc_fixed ? 0 : parc];
  rr_tile<T, CW, CH, BS>(a, w.y);
}

template <class T>
__global__ void k_prolong(const T* __restrict__ xc, int Nc, T* __restrict__ x, const uint8_t* __restrict__ fl,
                          const int* __restrict__ cutpos, T* __restrict__ snap, int s, int i0, int j0, int ni,
                          int nj) {
  const int ti = blockIdx.x * blockDim.x + threadIdx.x;
  const int tj = blockIdx.y * blockDim.y + threadIdx.y;
  if (ti >= ni || tj >= nj) return;
  const int i = i0 + ti, j = j0 + tj;
  const int64_t k = i + (int64_t)j * s;
  const uint8_t f = fl[k];
  if (!(f & kFlagActive)) return;
  const int sc = Nc + 1;
  const int64_t kc = (i >> 1) + (int64_t)(j >> 1) * sc;
  T val;
  if (!(i & 1) && !(j & 1)) val = xc[kc];
  else if ((i & 1) && !(j & 1)) val = T(0.5) * (xc[kc] + xc[kc + 1]);
  else if (!(i & 1) && (j & 1)) val = T(0.5) * (xc[kc] + xc[kc + sc]);
  else val = T(0.25) * ((xc[kc] + xc[kc + 1]) + (xc[kc + sc] + xc[kc + sc + 1]));
  const T v = x[k] + val;
  x[k] = v;
  if (f & kFlagCut) snap[cutpos[k]] = v;
}

template <class T>
__global__ void k_snap_gather(const int* __restrict__ list, int cnt, const T* __restrict__ x, T* __restrict__ snap) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < cnt) snap[q] = x[list[q]];
}

// ---------------------------------------------------------------------------
// Coarse levels in one workgroup.  Per level the host packs a descriptor of
// kDesc ints:
//   [0] N  [1] W  [2] H  [3] ox  [4] oy   LDS box: the bounding box grown by
//        one ring, W x H nodes with grid origin (ox, oy)
//   [5] first stored row in the global coefficient array (10 values per row:
//       8 off-diagonals in plane order 0,1,2,3,5,6,7,8, diagonal, 1/diagonal)
//   [6] first box node in the global slot array
//   [7..11] colour offsets of the cut list in the global cut-list array
//   [12..18] LDS byte offsets of x, b, r, active lists, slots, coefficients,
//            cut lists  [19] stored rows  [20] LDS offset of the coarsest inverse
//   [21..25] colour offsets of the active list in the global active-list array
// ---------------------------------------------------------------------------
template <class T>
struct CoarseArgs {
  const int* desc;
  const T* coef;
  const int16_t* slot;  // per box node: stored row, -1 interior Q1 row, -2 inactive
  const int16_t* cutl;
  const int16_t* actl;
  const double* inv;    // inverse of the coarsest active block
  const int16_t* cidx;  // coarsest active nodes as box indices
  const unsigned char* img;  // prebuilt static LDS block of all coarse levels
  int img_bytes;             // its size (whole 1 KB chunks)
  int lds_bytes;             // the whole LDS block (the vectors follow the image)
  int cn;
  int nlev;
  const T* b_top;
  T* x_top;
  int s_top;
  int nu1, nu2, eta, reverse, gstar;
  int reps;  // cycles of the first coarse level from its current iterate
  // column mode (set-up of the coarse map): workgroup j runs the cycles on the
  // unit right-hand side e_j (j-th node of the first coarse level's active
  // list) and writes the result into column j of map_out (row stride map_ld)
  int unit;
  T* map_out;
  int map_ld;
};

// pointers of one coarse level inside the LDS block
template <class T>
struct WgLev {
  int W, H, ox, oy;
  T* x;
  T* b;
  T* r;
  const int16_t* act;
  const int16_t* slot;
  const T* coef;
  const int16_t* cut;
  int act_off[5], cut_off[5];
  const double* inv;
};

template <class T>
__device__ inline WgLev<T> wg_level(const int* d, unsigned char* base) {
  WgLev<T> L;
  L.W = d[1];
  L.H = d[2];
  L.ox = d[3];
  L.oy = d[4];
  L.x = reinterpret_cast<T*>(base + d[12]);
  L.b = reinterpret_cast<T*>(base + d[13]);
  L.r = reinterpret_cast<T*>(base + d[14]);
  L.act = reinterpret_cast<const int16_t*>(base + d[15]);
  L.slot = reinterpret_cast<const int16_t*>(base + d[16]);
  L.coef = reinterpret_cast<const T*>(base + d[17]);
  L.cut = reinterpret_cast<const int16_t*>(base + d[18]);
  for (int c = 0; c < 5; ++c) {
    L.act_off[c] = d[21 + c] - d[21];
    L.cut_off[c] = d[7 + c] - d[7];
  }
  L.inv = reinterpret_cast<const double*>(base + d[20]);
  return L;
}

template <class T>
__device__ inline T lds_gs(const WgLev<T>& L, int q) {
  const int W = L.W;
  const T* x = L.x;
  const T bv = L.b[q];
  const int16_t sl = L.slot[q];
  if (sl >= 0) {
    const T* cf = L.coef + 10 * sl;
    const T acc = bv - (cf[0] * x[q - W - 1] + cf[1] * x[q - W] + cf[2] * x[q - W + 1] + cf[3] * x[q - 1] +
                        cf[4] * x[q + 1] + cf[5] * x[q + W - 1] + cf[6] * x[q + W] + cf[7] * x[q + W + 1]);
    return acc * cf[9];
  }
  const T nb = (x[q - W - 1] + x[q - W] + x[q - W + 1]) + (x[q - 1] + x[q + 1]) +
               (x[q + W - 1] + x[q + W] + x[q + W + 1]);
  return (T(3) * bv + nb) * T(0.125);
}

template <class T>
__device__ inline T lds_res(const WgLev<T>& L, int q) {
  const int W = L.W;
  const T* x = L.x;
  const T bv = L.b[q];
  const int16_t sl = L.slot[q];
  if (sl >= 0) {
    const T* cf = L.coef + 10 * sl;
    return bv - (cf[8] * x[q] + cf[0] * x[q - W - 1] + cf[1] * x[q - W] + cf[2] * x[q - W + 1] +
                 cf[3] * x[q - 1] + cf[4] * x[q + 1] + cf[5] * x[q + W - 1] + cf[6] * x[q + W] +
                 cf[7] * x[q + W + 1]);
  }
  const T nb = (x[q - W - 1] + x[q - W] + x[q - W + 1]) + (x[q - 1] + x[q + 1]) +
               (x[q + W - 1] + x[q + W] + x[q + W + 1]);
  return bv - (T(8) / T(3) * x[q] - nb * T(1.0 / 3.0));
}

// Gauss-Seidel value at q from a row slot and right-hand side held in registers
template <class T>
__device__ inline T lds_gs_reg(const WgLev<T>& L, int q, int16_t sl, T bv) {
  const int W = L.W;
  const T* x = L.x;
  if (sl >= 0) {
    const T* cf = L.coef + 10 * sl;
    const T acc = bv - (cf[0] * x[q - W - 1] + cf[1] * x[q - W] + cf[2] * x[q - W + 1] + cf[3] * x[q - 1] +
                        cf[4] * x[q + 1] + cf[5] * x[q + W - 1] + cf[6] * x[q + W] + cf[7] * x[q + W + 1]);
    return acc * cf[9];
  }
  const T nb = (x[q - W - 1] + x[q - W] + x[q - W + 1]) + (x[q - 1] + x[q + 1]) +
               (x[q + W - 1] + x[q + W] + x[q + W + 1]);
  return (T(3) * bv + nb) * T(0.125);
}

// nsteps smoothing steps of a level held in LDS.  Each thread first loads,
// for every colour of the full and the cut list, the index, row slot and
// right-hand side of its first kWgCache nodes into registers (once for all
// steps: they share the right-hand side); a colour phase then only reads x and
// the stored coefficients (independent LDS reads) before its barrier.  Nodes
// beyond the cached ones take the plain path.
constexpr int kWgCache = 2;

template <class T>
__device__ void wg_smooth(const WgLev<T>& L, int eta, bool reverse, int nsteps) {
  int qf[4][kWgCache], qc[4][kWgCache];
  int16_t sf[4][kWgCache], sc[4][kWgCache];
  T bf[4][kWgCache], bc[4][kWgCache];
  const int bs = blockDim.x, tid = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int u = 0; u < kWgCache; ++u) {
      const int tf = L.act_off[c] + tid + u * bs;
      const int q = tf < L.act_off[c + 1] ? L.act[tf] : -1;
      qf[c][u] = q;
      sf[c][u] = q >= 0 ? L.slot[q] : (int16_t)-1;
      bf[c][u] = q >= 0 ? L.b[q] : T(0);
      const int tc = L.cut_off[c] + tid + u * bs;
      const int r = tc < L.cut_off[c + 1] ? L.cut[tc] : -1;
      qc[c][u] = r;
      sc[c][u] = r >= 0 ? L.slot[r] : (int16_t)-1;
      bc[c][u] = r >= 0 ? L.b[r] : T(0);
    }
  auto full = [&](int c) {
#pragma unroll
    for (int u = 0; u < kWgCache; ++u)
      if (qf[c][u] >= 0) L.x[qf[c][u]] = lds_gs_reg<T>(L, qf[c][u], sf[c][u], bf[c][u]);
    for (int t = L.act_off[c] + tid + kWgCache * bs; t < L.act_off[c + 1]; t += bs) {
      const int q = L.act[t];
      L.x[q] = lds_gs<T>(L, q);
    }
    __syncthreads();
  };
  auto cut = [&](int c) {
#pragma unroll
    for (int u = 0; u < kWgCache; ++u)
      if (qc[c][u] >= 0) L.x[qc[c][u]] = lds_gs_reg<T>(L, qc[c][u], sc[c][u], bc[c][u]);
    for (int t = L.cut_off[c] + tid + kWgCache * bs; t < L.cut_off[c + 1]; t += bs) {
      const int q = L.cut[t];
      L.x[q] = lds_gs<T>(L, q);
    }
    __syncthreads();
  };
  for (int st = 0; st < nsteps; ++st) {
    if (!reverse) {
#pragma unroll
      for (int c = 0; c < 4; ++c) full(c);
      for (int e = 0; e < eta; ++e)
#pragma unroll
        for (int c = 0; c < 4; ++c) cut(c);
    } else {
      for (int e = 0; e < eta; ++e)
#pragma unroll
        for (int c = 3; c >= 0; --c) cut(c);
#pragma unroll
      for (int c = 3; c >= 0; --c) full(c);
    }
  }
}

// residual of level F restricted to level C (weights 1, 1/2, 1/4); x_C = 0
template <class T>
__device__ void wg_restrict(const WgLev<T>& F, const WgLev<T>& C) {
  const int na = F.act_off[4];
  for (int t = threadIdx.x; t < na; t += blockDim.x) {
    const int q = F.act[t];
    F.r[q] = lds_res<T>(F, q);
  }
  __syncthreads();
  const int nac = C.act_off[4];
  for (int t = threadIdx.x; t < nac; t += blockDim.x) {
    const int q = C.act[t];
    const int I = C.ox + q % C.W, J = C.oy + q / C.W;
    const int fi = 2 * I - F.ox, fj = 2 * J - F.oy;  // centre in the fine box
    T v = T(0);
    for (int dj = -1; dj <= 1; ++dj) {
      const int lj = fj + dj;
      if (lj < 0 || lj >= F.H) continue;
      const T wj = dj == 0 ? T(1) : T(0.5);
      const T* rr = F.r + lj * F.W;
      const T row = (fi >= 0 && fi < F.W) ? rr[fi] : T(0);
      T side = T(0);
      if (fi - 1 >= 0 && fi - 1 < F.W) side += rr[fi - 1];
      if (fi + 1 >= 0 && fi + 1 < F.W) side += rr[fi + 1];
      v += wj * (row + T(0.5) * side);
    }
    C.b[q] = v;
    C.x[q] = T(0);
  }
  __syncthreads();
}

template <class T>
__device__ void wg_prolong(const WgLev<T>& F, const WgLev<T>& C) {
  const int na = F.act_off[4];
  const int Wc = C.W;
  for (int t = threadIdx.x; t < na; t += blockDim.x) {
    const int q = F.act[t];
    const int i = F.ox + q % F.W, j = F.oy + q / F.W;
    const int kc = ((i >> 1) - C.ox) + ((j >> 1) - C.oy) * Wc;
    const T* xc = C.x;
    T val;
    if (!(i & 1) && !(j & 1)) val = xc[kc];
    else if ((i & 1) && !(j & 1)) val = T(0.5) * (xc[kc] + xc[kc + 1]);
    else if (!(i & 1) && (j & 1)) val = T(0.5) * (xc[kc] + xc[kc + Wc]);
    else val = T(0.25) * ((xc[kc] + xc[kc + 1]) + (xc[kc + Wc] + xc[kc + Wc + 1]));
    F.x[q] += val;
  }
  __syncthreads();
}

constexpr int kMaxWgLevels = 12;

// One cycle from the first coarse level, written without recursion (a
// recursive device function would keep its frames in scratch memory).  The
// counters of coarse-grid visits (gamma* per level) live in a 64-bit word.
template <class T>
__device__ void wg_cycle(const CoarseArgs<T>& a, const int* sdesc, unsigned char* base) {
  const int last = a.nlev - 1;
  const int pre = a.reverse ? a.nu2 : a.nu1, post = a.reverse ? a.nu1 : a.nu2;
  unsigned long long visits = 0;  // 4 bits per level
  int l = 0;
  bool enter = true;
  while (l >= 0) {
    if (enter) {
      const WgLev<T> L = wg_level<T>(sdesc + kDesc * l, base);
      if (l == last) {  // exact solve with the stored inverse (float64)
        for (int r = threadIdx.x; r < a.cn; r += blockDim.x) {
          double acc = 0.0;
          for (int cc = 0; cc < a.cn; ++cc) acc += L.inv[r * a.cn + cc] * (double)L.b[L.act[cc]];
          L.x[L.act[r]] = (T)acc;
        }
        __syncthreads();
        enter = false;
        --l;
        continue;
      }
      const WgLev<T> C = wg_level<T>(sdesc + kDesc * (l + 1), base);
      wg_smooth<T>(L, a.eta, a.reverse, pre);
      wg_restrict<T>(L, C);
      visits &= ~(0xfull << (4 * l));
      ++l;
      continue;
    }
    const unsigned long long g = ((visits >> (4 * l)) & 0xf) + 1;
    visits = (visits & ~(0xfull << (4 * l))) | (g << (4 * l));
    if ((int)g < a.gstar) {  // another coarse-grid cycle from the current iterate
      ++l;
      enter = true;
      continue;
    }
    const WgLev<T> L = wg_level<T>(sdesc + kDesc * l, base);
    const WgLev<T> C = wg_level<T>(sdesc + kDesc * (l + 1), base);
    wg_prolong<T>(L, C);
    wg_smooth<T>(L, a.eta, a.reverse, post);
    --l;
  }
}

// stage every coarse level into LDS, run gamma* cycles, write the first coarse
// level's iterate back to global memory (ends with a barrier)
template <class T>
__device__ void coarse_body(const CoarseArgs<T>& a, unsigned char* base, int* sdesc) {
  for (int q = threadIdx.x; q < kDesc * a.nlev; q += blockDim.x) sdesc[q] = a.desc[q];
  // the static LDS block of every coarse level (lists, slots, rows, the
  // coarsest inverse) comes from a prebuilt image with global->LDS loads of
  // 16 bytes per lane, all in flight together; the vectors are zeroed
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int ch = wave; ch < (a.img_bytes >> 10); ch += nw)
      __builtin_amdgcn_global_load_lds(a.img + ch * 1024 + lane * 16,
                                       (__attribute__((address_space(3))) void*)(base + ch * 1024), 16, 0, 0);
    uint4* vz = reinterpret_cast<uint4*>(base + a.img_bytes);
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int q = threadIdx.x; q < ((a.lds_bytes - a.img_bytes) >> 4); q += blockDim.x) vz[q] = z;
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  // right-hand side of the first coarse level at its active nodes
  if (a.unit) {
    const WgLev<T> L = wg_level<T>(sdesc, base);
    if (threadIdx.x == 0) L.b[L.act[blockIdx.x]] = T(1);
  } else {
    const WgLev<T> L = wg_level<T>(sdesc, base);
    const int na = L.act_off[4];
    for (int t0 = 0; t0 < na; t0 += 8 * (int)blockDim.x) {
      T v[8];
      int qq[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + (int)threadIdx.x + u * (int)blockDim.x;
        qq[u] = t < na ? L.act[t] : -1;
        if (qq[u] >= 0) {
          const int gi = L.ox + qq[u] % L.W, gj = L.oy + qq[u] / L.W;
          v[u] = a.b_top[gi + (int64_t)gj * a.s_top];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (qq[u] >= 0) L.b[qq[u]] = v[u];
    }
  }
  __syncthreads();
  // reps cycles on the first coarse level, each continuing from the last
  for (int g = 0; g < a.reps; ++g) wg_cycle<T>(a, sdesc, base);
  const WgLev<T> L = wg_level<T>(sdesc, base);
  if (a.unit) {
    for (int t = threadIdx.x; t < L.act_off[4]; t += blockDim.x)
      a.map_out[(int64_t)t * a.map_ld + blockIdx.x] = L.x[L.act[t]];
    __syncthreads();
    return;
  }
  for (int t = threadIdx.x; t < L.act_off[4]; t += blockDim.x) {
    const int q = L.act[t];
    const int gi = L.ox + q % L.W, gj = L.oy + q / L.W;
    a.x_top[gi + (int64_t)gj * a.s_top] = L.x[q];
  }
  __syncthreads();
}

template <class T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse(CoarseArgs<T> a) {
  extern __shared__ __align__(16) unsigned char base[];
  __shared__ int sdesc[kDesc * kMaxWgLevels];
  coarse_body<T>(a, base, sdesc);
}

// The coarse part of a cycle as one dense product.  From a zero start the
// cycles that k_coarse runs on the first coarse level (pre-smoothing,
// restriction, the levels below, prolongation, post-smoothing, each a linear
// step) map its right-hand side b to x = B b with a fixed matrix B, computed
// at set-up by running those cycles on every unit vector.  Applying B reads
// n^2 values with all CUs instead of running the ~250 barrier-separated
// phases of the single-workgroup cycle.  One wave per row of B: the row is
// loaded with 16-byte loads before b is gathered into LDS, then reduced
// across the wave.
template <class T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
  __device__ static double dot(const double2& v, const double* s) { return v.x * s[0] + v.y * s[1]; }
};
template <>
struct Vec16<float> {
  using type = float4;
  __device__ static float dot(const float4& v, const float* s) {
    return (v.x * s[0] + v.y * s[1]) + (v.z * s[2] + v.w * s[3]);
  }
};

constexpr int kMapWaves = 4;  // rows of B per 256-thread workgroup

template <class T>
struct MapEntry {
  const T* B;
  int ld;
  const int* idx;
  int n;
  const T* b;
  T* x;
};

// rows kMapWaves blk ... kMapWaves (blk + 1) - 1 of x = B b (sb: ld values of LDS)
template <class T>
__device__ __forceinline__ void map_rows(const T* __restrict__ B, int ld, const int* __restrict__ idx, int n,
                         const T* __restrict__ b, T* __restrict__ x, const int blk, T* sb) {
  using V = typename Vec16<T>::type;
  constexpr int G = 16 / (int)sizeof(T);  // values per 16-byte load
  constexpr int U = 4;                    // loads per lane and round; two rounds in flight
  constexpr int CH = U * 64 * G;          // values of a row per round
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = blk * kMapWaves + wave;
  const T* row = B + (int64_t)(r < n ? r : 0) * ld;
  // two rounds of the row in flight at a time (double-buffered registers)
  V v0[U], v1[U];
  auto load = [&](V* v, int base) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int col = base + (u * 64 + lane) * G;
      v[u] = col < ld ? *reinterpret_cast<const V*>(row + col) : V{};
    }
  };
  T acc = T(0);
  auto dot = [&](const V* v, int base) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int col = base + (u * 64 + lane) * G;
      if (col < ld) acc += Vec16<T>::dot(v[u], sb + col);
    }
  };
  load(v0, 0);
  load(v1, CH);
  // b gathered into LDS, GC values per thread at a time with all their loads
  // in flight: the indices, then the values (n >= 1)
  {
    constexpr int NT = 64 * kMapWaves, GC = 8;
    for (int j0 = 0; j0 < ld; j0 += GC * NT) {
      int ii[GC];
#pragma unroll
      for (int u = 0; u < GC; ++u) {
        const int j = j0 + (int)threadIdx.x + u * NT;
        ii[u] = idx[j < n ? j : n - 1];
      }
      T bv[GC];
#pragma unroll
      for (int u = 0; u < GC; ++u) bv[u] = b[ii[u]];
#pragma unroll
      for (int u = 0; u < GC; ++u) {
        const int j = j0 + (int)threadIdx.x + u * NT;
        if (j < ld) sb[j] = j < n ? bv[u] : T(0);
      }
    }
  }
  __syncthreads();
  for (int base = 0; base < ld; base += 2 * CH) {
    dot(v0, base);
    if (base + 2 * CH < ld) load(v0, base + 2 * CH);
    if (base + CH < ld) dot(v1, base + CH);
    if (base + 3 * CH < ld) load(v1, base + 3 * CH);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0 && r < n) x[idx[r]] = acc;
}

template <class T>
__global__ __launch_bounds__(64 * kMapWaves) void k_coarse_apply(const T* __restrict__ B, int ld,
                                                                 const int* __restrict__ idx, int n,
                                                                 const T* __restrict__ b, T* __restrict__ x) {
  extern __shared__ __align__(16) unsigned char smem[];
  map_rows<T>(B, ld, idx, n, b, x, blockIdx.x, reinterpret_cast<T*>(smem));
}

template <class T>
__global__ __launch_bounds__(64 * kMapWaves) void k_coarse_apply_multi(const MapEntry<T>* tab, const int2* work,
                                                                       int nwork) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int i = blockIdx.x;
  if (i >= nwork) return;
  const int2 w = work[i];
  const MapEntry<T>& E = tab[w.x];
  map_rows<T>(E.B, E.ld, E.idx, E.n, E.b, E.x, w.y, reinterpret_cast<T*>(smem));
}

__global__ void k_f64_to_f32(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) d[q] = (float)s[q];
}

inline unsigned nblk(int64_t n, int tb) { return (unsigned)((n + tb - 1) / tb); }

template <class T>
T* Xp(Level& L, int which);
template <>
double* Xp<double>(Level& L, int which) { return L.X[which]; }
template <>
float* Xp<float>(Level& L, int which) { return L.X32[which]; }
template <class T>
T* Bp(Level& L);
template <>
double* Bp<double>(Level& L) { return L.b; }
template <>
float* Bp<float>(Level& L) { return L.b32; }
template <class T>
const T* Ap(Level& L);
template <>
const double* Ap<double>(Level& L) { return L.A; }
template <>
const float* Ap<float>(Level& L) { return L.A32; }
template <class T>
T* Sp(Level& L);
template <>
double* Sp<double>(Level& L) { return L.snap; }
template <>
float* Sp<float>(Level& L) { return L.snap32; }

// arguments of the sweep of level l with TW x TH tiles from the level's
// current state (ping-pong parities)
template <class T, int TW, int TH>
SweepArgs<T> sweep_args(mgfem_ctx* c, int l, bool reverse, bool norm, bool prolong_from) {
  Level& L = c->lv[l];
  SweepArgs<T> a;
  a.part = c->sweep_part;
  a.norm = norm ? 1 : 0;
  a.xc = nullptr;
  a.sc = 0;
  if (prolong_from) {
    Level& C = c->lv[l + 1];
    a.xc = Xp<T>(C, C.cur);
    a.sc = C.stride;
  }
  a.xin = Xp<T>(L, L.cur);
  a.xout = Xp<T>(L, 1 - L.cur);
  a.b = Bp<T>(L);
  a.A = Ap<T>(L);
  a.fl = L.flags;
  a.cutpos = L.cutpos;
  a.snap = Sp<T>(L);
  a.N = L.N;
  a.s = L.stride;
  a.n = L.n;
  a.i0 = L.bbox[0];
  a.i1 = L.bbox[1];
  a.j0 = L.bbox[2];
  a.j1 = L.bbox[3];
  a.ntx = (a.i1 - a.i0 + TW) / TW;
  a.nty = (a.j1 - a.j0 + TH) / TH;
  // the tile list and its plans exist for every level with a smoother, in
  // the shape sweep_shape() gives
  a.tiles = L.tiles;
  a.ntiles = L.ntiles;
  a.per = (a.ntiles + 7) / 8;
  a.reverse = reverse ? 1 : 0;
  a.tmeta = L.tmeta;
  a.tp_off = L.tp_off;
  a.tp_idx = L.tp_idx;
  a.tp_coef = std::is_same<T, double>::value ? reinterpret_cast<const T*>(L.tp_coef)
                                             : reinterpret_cast<const T*>(L.tp_coef32);
  a.tc_off = L.tc_off;
  a.tc_idx = L.tc_idx;
  a.tc_pos = L.tc_pos;
  a.zero = reinterpret_cast<const T*>(c->zero);
  return a;
}

template <class T, int TW, int TH, int BS>
void launch_sweep(mgfem_ctx* c, int l, bool reverse, bool norm, bool prolong_from, int shape) {
  Level& L = c->lv[l];
  const SweepArgs<T> a = sweep_args<T, TW, TH>(c, l, reverse, norm, prolong_from);
  (void)shape;
  if (c->prof.on && l == 0) {
    // algorithmic bytes (matrix-free interior rows): per active row x read
    // and written and b read, the nine coefficients of a stored row; a fused
    // prolongation also reads x_c (class 0 float64, class 1 the float32
    // sweeps of the mixed solve).  The flag byte per node is not counted.
    // Every launch is idempotent (it reads one iterate buffer and writes the
    // other), so a profiled launch may be repeated back to back.
    constexpr double vb = (double)sizeof(T);
    double bytes = 3.0 * vb * L.n_active + 9.0 * vb * L.n_stored;
    if (prolong_from) bytes += vb * c->lv[l + 1].n_active;
    prof_launch(c, std::is_same<T, double>::value ? 0 : 1, bytes, [a](hipStream_t st) {
      hipLaunchKernelGGL((k_sweep<T, TW, TH, BS>), dim3(8 * a.per), dim3(BS), 0, st, a);
    });
  } else {
    hipLaunchKernelGGL((k_sweep<T, TW, TH, BS>), dim3(8 * a.per), dim3(BS), 0, c->s, a);
  }
  if (norm) {
    c->red_seq += 1.0;
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(1024), 0, c->s, (const double*)c->sweep_part, a.ntiles,
                       c->red_out, c->red_host, c->red_seq_dev);
  }
  L.cur = 1 - L.cur;
}

template <class T>
void sweep(mgfem_ctx* c, int l, bool reverse, bool norm = false, bool prolong_from = false) {
  Level& L = c->lv[l];
  if (L.empty()) return;
  switch (sweep_shape(c, l)) {
    case kShapeFinest: launch_sweep<T, 64, 32, 512>(c, l, reverse, norm, prolong_from, kShapeFinest); break;
    case kShapeLarge: launch_sweep<T, 64, 16, 512>(c, l, reverse, norm, prolong_from, kShapeLarge); break;
    default: launch_sweep<T, 16, 16, 512>(c, l, reverse, norm, prolong_from, kShapeSmall); break;
  }
}

template <class T>
CutArgs<T> cut_args(mgfem_ctx* c, int l, bool reverse) {
  Level& L = c->lv[l];
  CutArgs<T> a;
  a.g_info = L.cp.g_info;
  a.cl_node = L.cp.cl_node;
  a.cl_q = L.cp.cl_q;
  a.cl_own = L.cp.cl_own;
  a.cl_nbr = L.cp.cl_nbr;
  a.ext_src = L.cp.ext_src;
  a.cl_coef = std::is_same<T, double>::value ? reinterpret_cast<const T*>(L.cp.cl_coef)
                                             : reinterpret_cast<const T*>(L.cp.cl_coef32);
  a.x = Xp<T>(L, L.cur);
  a.b = Bp<T>(L);
  a.snap = Sp<T>(L);
  a.eta = c->p.eta;
  a.reverse = reverse ? 1 : 0;
  return a;
}

template <class T>
void cut_sweeps(mgfem_ctx* c, int l, bool reverse) {
  Level& L = c->lv[l];
  const int eta = c->p.eta;
  if (eta == 0 || L.cut_off[4] == 0) return;
  if (L.cp.ok) {
    const CutArgs<T> a = cut_args<T>(c, l, reverse);
    const size_t lds = std::is_same<T, double>::value ? L.cp.lds64 : L.cp.lds32;
    hipLaunchKernelGGL(k_cut<T>, dim3(L.cp.ngroups), dim3(kCutThreads), lds, c->s, a);
    return;
  }
  for (int e = 0; e < eta; ++e)
    for (int p = 0; p < 4; ++p) {
      const int col = reverse ? 3 - p : p;
      const int cnt = L.cut_off[col + 1] - L.cut_off[col];
      if (cnt <= 0) continue;
      hipLaunchKernelGGL(k_gs_list<T>, dim3(nblk(cnt, 256)), dim3(256), 0, c->s, Ap<T>(L), L.flags,
                         Xp<T>(L, L.cur), (const T*)Bp<T>(L), L.N, L.n, L.cut_list + L.cut_off[col], cnt);
    }
}

template <class T>
void smooth(mgfem_ctx* c, int l, bool reverse) {
  if (!reverse) {
    sweep<T>(c, l, false);
    cut_sweeps<T>(c, l, false);
  } else {
    cut_sweeps<T>(c, l, true);
    sweep<T>(c, l, true);
  }
}

template <class T, int CW, int CH>
ResArgs<T> rr_args(mgfem_ctx* c, int l) {
  Level& L = c->lv[l];
  Level& C = c->lv[l + 1];
  ResArgs<T> a;
  a.x = Xp<T>(L, L.cur);
  a.b = Bp<T>(L);
  a.A = Ap<T>(L);
  a.fl = L.flags;
  a.N = L.N;
  a.s = L.stride;
  a.n = L.n;
  a.bc = Bp<T>(C);
  a.xc = Xp<T>(C, C.cur);
  a.flc = C.flags;
  a.cutposc = C.cutpos;
  a.snapc = Sp<T>(C);
  a.Nc = C.N;
  a.sc = C.stride;
  a.I0 = C.bbox[0];
  a.I1 = C.bbox[1];
  a.J0 = C.bbox[2];
  a.J1 = C.bbox[3];
  a.ntx = (a.I1 - a.I0 + CW) / CW;
  a.nty = (a.J1 - a.J0 + CH) / CH;
  a.tiles = L.rr_tiles;
  a.ntiles = L.rr_ntiles;
  a.per = (a.ntiles + 7) / 8;
  return a;
}

template <class T, int CW, int CH, int BS>
void launch_resrestrict(mgfem_ctx* c, int l) {
  Level& L = c->lv[l];
  Level& C = c->lv[l + 1];
  if (C.empty() || L.rr_ntiles == 0) return;
  const ResArgs<T> a = rr_args<T, CW, CH>(c, l);
  hipLaunchKernelGGL((k_resrestrict<T, CW, CH, BS>), dim3(8 * a.per), dim3(BS), 0, c->s, a);
}

template <class T>
void prolong(mgfem_ctx* c, int l) {
  Level& L = c->lv[l];
  Level& C = c->lv[l + 1];
  if (L.empty()) return;
  const int ni = L.bbox[1] - L.bbox[0] + 1, nj = L.bbox[3] - L.bbox[2] + 1;
  dim3 grid(nblk(ni, 64), nblk(nj, 4));
  hipLaunchKernelGGL(k_prolong<T>, grid, dim3(64, 4), 0, c->s, (const T*)Xp<T>(C, C.cur), C.N,
                     Xp<T>(L, L.cur), L.flags, L.cutpos, Sp<T>(L), L.stride, L.bbox[0], L.bbox[2], ni, nj);
}

// arguments of k_coarse for `reps` cycles of the coarse part
template <class T>
CoarseArgs<T> coarse_args(mgfem_ctx* c, bool reverse, int reps) {
  CoarsePlan& P = c->cplan;
  Level& Lc = c->lv[P.lc];
  CoarseArgs<T> a;
  const bool f32 = !std::is_same<T, double>::value;
  a.desc = P.desc + (f32 ? kDesc * P.ndesc : 0);
  a.coef = std::is_same<T, double>::value ? reinterpret_cast<const T*>(P.coef)
                                          : reinterpret_cast<const T*>(P.coef32);
  a.slot = P.slot;
  a.cutl = P.cutl;
  a.actl = P.actl;
  a.inv = P.inv;
  a.cidx = nullptr;
  a.img = f32 ? P.img32 : P.img64;
  a.img_bytes = f32 ? P.static32 : P.static64;
  a.lds_bytes = f32 ? P.lds32 : P.lds64;
  a.cn = c->coarse_n;
  a.nlev = P.ndesc;
  a.b_top = Bp<T>(Lc);
  a.x_top = Xp<T>(Lc, 0);
  a.s_top = Lc.stride;
  a.nu1 = c->p.nu1;
  a.nu2 = c->p.nu2;
  a.eta = c->p.eta;
  a.reverse = reverse ? 1 : 0;
  a.gstar = c->p.cycle == MGFEM_CYCLE_W ? 2 : 1;
  a.reps = reps;
  a.unit = 0;
  a.map_out = nullptr;
  a.map_ld = 0;
  return a;
}

template <class T>
const T* coarse_map(const CoarseMap& M, bool reverse);
template <>
const double* coarse_map<double>(const CoarseMap& M, bool reverse) { return M.f64[reverse ? 1 : 0]; }
template <>
const float* coarse_map<float>(const CoarseMap& M, bool reverse) { return reverse ? nullptr : M.f32; }

// the first level of a cycle's coarse part: where the coarse map applies,
// else the single-workgroup part
inline int coarse_level(const mgfem_ctx* c) {
  return c->cplan.map.level >= 0 ? c->cplan.map.level : c->cplan.lc;
}

template <class T>
void coarse_wg(mgfem_ctx* c, bool reverse, int reps) {
  CoarsePlan& P = c->cplan;
  const T* B = coarse_map<T>(P.map, reverse);
  if (B && reps == P.map.reps) {
    Level& Lc = c->lv[P.map.level];
    const int n = P.map.n;
    hipLaunchKernelGGL(k_coarse_apply<T>, dim3(nblk(n, kMapWaves)), dim3(64 * kMapWaves),
                       P.map.ld * sizeof(T), c->s, B, P.map.ld, (const int*)P.map.idx, n,
                       (const T*)Bp<T>(Lc), Xp<T>(Lc, 0));
    Lc.cur = 0;
    return;
  }
  Level& Lc = c->lv[P.lc];
  const CoarseArgs<T> a = coarse_args<T>(c, reverse, reps);
  const int lds = std::is_same<T, double>::value ? P.lds64 : P.lds32;
  hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(kCoarseThreads), lds, c->s, a);
  Lc.cur = 0;
}

template <class T>
void cycle_level(mgfem_ctx* c, int l, bool reverse, bool first_sweep_done = false) {
  const int nl = (int)c->lv.size();
  const int cl = coarse_level(c);
  if (cl >= 0 && l == cl) {
    coarse_wg<T>(c, reverse, 1);
    return;
  }
  if (l == nl - 1) return;  // unreachable: the coarse plan always covers the coarsest level
  const int pre = reverse ? c->p.nu2 : c->p.nu1;
  const int post = reverse ? c->p.nu1 : c->p.nu2;
  for (int s = 0; s < pre; ++s) {
    if (s == 0 && first_sweep_done) cut_sweeps<T>(c, l, reverse);
    else smooth<T>(c, l, reverse);
  }
  if (c->lv[l].N >= 1024) launch_resrestrict<T, 32, 16, 512>(c, l);
  else launch_resrestrict<T, 16, 8, 512>(c, l);
  // coarse-grid visits: gamma* (section 3.2); the two-grid scheme instead
  // solves the first coarse problem with coarse_cycles V-cycles from zero
  const bool two_grid = c->p.cycle == MGFEM_CYCLE_TWO_GRID && l == 0;
  const int visits = two_grid ? c->p.coarse_cycles : (c->p.cycle == MGFEM_CYCLE_W ? 2 : 1);
  if (l + 1 == cl) coarse_wg<T>(c, reverse, visits);  // runs its visits itself
  else
    for (int g = 0; g < visits; ++g) cycle_level<T>(c, l + 1, reverse);
  if (reverse || post == 0) {
    prolong<T>(c, l);
    for (int s = 0; s < post; ++s) smooth<T>(c, l, reverse);
  } else {
    sweep<T>(c, l, false, false, true);  // x + P x_c, then the sweep
    cut_sweeps<T>(c, l, false);
    for (int s = 1; s < post; ++s) smooth<T>(c, l, reverse);
  }
}

}  // namespace

void run_cycle(mgfem_ctx* c, const CycleOpts& o) {
  if (o.fp32) cycle_level<float>(c, 0, o.reverse, o.first_sweep_done);
  else cycle_level<double>(c, 0, o.reverse, o.first_sweep_done);
}

void first_sweep_with_norm(mgfem_ctx* c) { sweep<double>(c, 0, false, true); }

// ---- batched solves on the tiled kernels: float-cycle entries and launches.
// Every level a batch member smooths must use the small tile shapes (16 x 16
// sweep tiles, 16 x 8 residual tiles) and have its cut groups; the first
// level of its coarse part is applied with its float map.
size_t team_entry_bytes(int kind) {
  switch (kind) {
    case kTeamSweep: return sizeof(SweepEntry<float>);
    case kTeamCut: return sizeof(CutEntry<float>);
    case kTeamRR: return sizeof(RrEntry<float>);
    case kTeamMap: return sizeof(MapEntry<float>);
  }
  return 0;
}

void team_entry(mgfem_ctx* m, int kind, int l, void* out) {
  Level& L = m->lv[l];
  const bool fixed = m->cplan.lc == l + 1;  // the coarser level is the coarse map's level
  switch (kind) {
    case kTeamSweep: {
      SweepEntry<float> e{};
      e.a = sweep_args<float, 16, 16>(m, l, false, false, false);
      e.a.sc = m->lv[l + 1].stride;
      e.X[0] = L.X32[0];
      e.X[1] = L.X32[1];
      e.XC[0] = m->lv[l + 1].X32[0];
      e.XC[1] = m->lv[l + 1].X32[1];
      e.xc_fixed = fixed ? 1 : 0;
      std::memcpy(out, &e, sizeof e);
      break;
    }
    case kTeamCut: {
      CutEntry<float> e{};
      if (L.cp.ok) e.a = cut_args<float>(m, l, false);
      e.X[0] = L.X32[0];
      e.X[1] = L.X32[1];
      std::memcpy(out, &e, sizeof e);
      break;
    }
    case kTeamRR: {
      RrEntry<float> e{};
      e.a = rr_args<float, 16, 8>(m, l);
      e.X[0] = L.X32[0];
      e.X[1] = L.X32[1];
      e.XC[0] = m->lv[l + 1].X32[0];
      e.XC[1] = m->lv[l + 1].X32[1];
      e.xc_fixed = fixed ? 1 : 0;
      std::memcpy(out, &e, sizeof e);
      break;
    }
    case kTeamMap: {
      MapEntry<float> e{};
      const CoarseMap& M = m->cplan.map;
      Level& Lc = m->lv[m->cplan.lc];
      e.B = M.f32;
      e.ld = M.ld;
      e.idx = M.idx;
      e.n = M.n;
      e.b = Lc.b32;
      e.x = Lc.X32[0];
      std::memcpy(out, &e, sizeof e);
      break;
    }
  }
}

int team_units(mgfem_ctx* m, int kind, int l) {
  Level& L = m->lv[l];
  switch (kind) {
    case kTeamSweep:
      if (L.empty()) return 0;
      return sweep_shape(m, l) == kShapeSmall ? L.ntiles : -1;
    case kTeamCut:
      if (m->p.eta == 0 || L.cut_off[4] == 0) return 0;
      return L.cp.ok ? L.cp.ngroups : -1;
    case kTeamRR:
      if (m->lv[l + 1].empty()) return 0;
      return L.N < 1024 ? L.rr_ntiles : -1;
    case kTeamMap: {
      const CoarseMap& M = m->cplan.map;
      if (M.n <= 0) return 0;
      return M.f32 && M.reps == 1 ? (M.n + kMapWaves - 1) / kMapWaves : -1;
    }
  }
  return -1;
}

int team_lds(mgfem_ctx* m, int kind, int l) {
  if (kind == kTeamCut) return m->lv[l].cp.lds32;
  if (kind == kTeamMap) return m->cplan.map.ld * (int)sizeof(float);
  return 0;
}

void team_launch(hipStream_t s, int kind, const void* tab, const int2* work, int nwork, int par, int parc,
                 int prolong, int lds) {
  if (nwork <= 0) return;
  const unsigned grid = 8u * (unsigned)((nwork + 7) / 8);
  switch (kind) {
    case kTeamSweep:
      hipLaunchKernelGGL((k_sweep_multi<float, 16, 16, 512>), dim3(grid), dim3(512), 0, s,
                         static_cast<const SweepEntry<float>*>(tab), work, nwork, par, parc, prolong);
      break;
    case kTeamCut:
      hipLaunchKernelGGL(k_cut_multi<float>, dim3(grid), dim3(kCutThreads), lds, s, static_cast<const CutEntry<float>*>(tab),
                         work, nwork, par);
      break;
    case kTeamRR:
      hipLaunchKernelGGL((k_resrestrict_multi<float, 16, 8, 512>), dim3(grid), dim3(512), 0, s,
                         static_cast<const RrEntry<float>*>(tab), work, nwork, par, parc);
      break;
    case kTeamMap:
      hipLaunchKernelGGL(k_coarse_apply_multi<float>, dim3(nwork), dim3(64 * kMapWaves), lds, s,
                         static_cast<const MapEntry<float>*>(tab), work, nwork);
      break;
  }
}

// tile activity of one level for its sweep shape: a tile is kept when its core
// holds an active node (tiles entirely outside the domain are skipped)
__global__ void k_tile_active(const uint8_t* __restrict__ fl, int s, int i0, int j0, int i1, int j1, int TW, int TH,
                              int ntx, int nty, int* __restrict__ act) {
  const int t = blockIdx.x;
  if (t >= ntx * nty) return;
  const int x0 = i0 + (t % ntx) * TW, y0 = j0 + (t / ntx) * TH;
  int any = 0;
  for (int q = threadIdx.x; q < TW * TH; q += blockDim.x) {
    const int gi = x0 + q % TW, gj = y0 + q / TW;
    if (gi <= i1 && gj <= j1 && (fl[gi + (int64_t)gj * s] & kFlagActive)) any = 1;
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) act[t] = any;
}

// Tile plan of one sweep tile (one block per tile in list order): the stored
// rows of its phase-0 box (the staged region less its outer ring) and the cut
// vertices of its core.  fill = 0 counts, fill = 1 writes the entries at the
// offsets (order within a tile is free: updates of one colour are independent).
__global__ void k_tile_plan(const uint8_t* __restrict__ fl, const double* __restrict__ A,
                            const float* __restrict__ A32, int64_t n, const int* __restrict__ cutpos, int N, int s,
                            int i0, int j0, int i1, int j1, int TW, int TH, int ntx,
                            const int* __restrict__ tiles, int fill, int* __restrict__ cnt,
                            int* __restrict__ ccnt, const int* __restrict__ off, const int* __restrict__ coff,
                            int* __restrict__ idx, double* __restrict__ coef, float* __restrict__ coef32,
                            int* __restrict__ cidx, int* __restrict__ cpos) {
  __shared__ int nr, nc;
  if (threadIdx.x == 0) nr = nc = 0;
  __syncthreads();
  const int t = blockIdx.x;
  const int tile = tiles[t];
  const int RW = TW + 2 * kHalo, RH = TH + 2 * kHalo;
  const int ox = i0 + (tile % ntx) * TW - kHalo, oy = j0 + (tile / ntx) * TH - kHalo;
  for (int q = threadIdx.x; q < RW * RH; q += blockDim.x) {
    const int ri = q % RW, rj = q / RW;
    const int gi = ox + ri, gj = oy + rj;
    if (ri < 1 || rj < 1 || ri >= RW - 1 || rj >= RH - 1 || gi < 0 || gj < 0 || gi > N || gj > N) continue;
    const int64_t k = gi + (int64_t)gj * s;
    const uint8_t f = fl[k];
    if ((f & kFlagActive) && (f & kFlagStored)) {
      const int e = atomicAdd(&nr, 1);
      if (fill) {
        const int64_t w = off[t] + e;
        idx[w] = q;
        for (int p = 0; p < 9; ++p) coef[9 * w + p] = A[p * n + k];
        if (coef32)
          for (int p = 0; p < 9; ++p) coef32[9 * w + p] = A32[p * n + k];
      }
    }
    const bool core = ri >= kHalo && ri < kHalo + TW && rj >= kHalo && rj < kHalo + TH && gi <= i1 && gj <= j1;
    if (core && (f & kFlagCut)) {
      const int e = atomicAdd(&nc, 1);
      if (fill) {
        cidx[coff[t] + e] = q;
        cpos[coff[t] + e] = cutpos[k];
      }
    }
  }
  __syncthreads();
  if (!fill && threadIdx.x == 0) {
    cnt[t] = nr;
    ccnt[t] = nc;
  }
}

int build_tile_lists(mgfem_ctx* c) {
  const int nl = (int)c->lv.size();
  for (int l = 0; l + 1 < nl; ++l) {  // every level with a smoother
    Level& L = c->lv[l];
    if (L.empty()) continue;
    const int shape = sweep_shape(c, l);
    const int TW = shape == kShapeSmall ? 16 : 64;
    const int TH = shape == kShapeFinest ? 32 : 16;
    const int ntx = (L.bbox[1] - L.bbox[0] + TW) / TW, nty = (L.bbox[3] - L.bbox[2] + TH) / TH;
    int* act = nullptr;
    MGFEM_HIP_TRY(ctx_alloc_t(c, &act, ntx * nty));
    hipLaunchKernelGGL(k_tile_active, dim3(ntx * nty), dim3(256), 0, c->s, L.flags, L.stride, L.bbox[0], L.bbox[2],
                       L.bbox[1], L.bbox[3], TW, TH, ntx, nty, act);
    std::vector<int> h(ntx * nty);
    MGFEM_HIP_TRY(hipMemcpyAsync(h.data(), act, h.size() * sizeof(int), hipMemcpyDeviceToHost, c->s));
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
    std::vector<int> list;
    for (int t = 0; t < ntx * nty; ++t)
      if (h[t]) list.push_back(t);
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.tiles, std::max<size_t>(1, list.size())));
    if (!list.empty())
      MGFEM_HIP_TRY(hipMemcpyAsync(L.tiles, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice, c->s));
    L.ntiles = (int)list.size();
    L.tile_shape = shape;
    // tile plans: count, offsets, fill
    const int nt = L.ntiles;
    int *cnt = nullptr, *ccnt = nullptr;
    MGFEM_HIP_TRY(ctx_alloc_t(c, &cnt, std::max(1, nt)));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &ccnt, std::max(1, nt)));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.tp_off, nt + 1));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.tc_off, nt + 1));
    if (nt > 0)
      hipLaunchKernelGGL(k_tile_plan, dim3(nt), dim3(256), 0, c->s, L.flags, L.A, L.A32, L.n, L.cutpos, L.N,
                         L.stride, L.bbox[0], L.bbox[2], L.bbox[1], L.bbox[3], TW, TH, ntx, L.tiles, 0, cnt, ccnt,
                         nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    MGFEM_HIP_TRY(hipGetLastError());
    std::vector<int> hc(std::max(1, nt)), hcc(std::max(1, nt)), ho(nt + 1), hco(nt + 1);
    MGFEM_HIP_TRY(hipMemcpyAsync(hc.data(), cnt, hc.size() * sizeof(int), hipMemcpyDeviceToHost, c->s));
    MGFEM_HIP_TRY(hipMemcpyAsync(hcc.data(), ccnt, hcc.size() * sizeof(int), hipMemcpyDeviceToHost, c->s));
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
    ho[0] = hco[0] = 0;
    L.tp_max = L.tc_max = 0;
    for (int q = 0; q < nt; ++q) {
      ho[q + 1] = ho[q] + hc[q];
      hco[q + 1] = hco[q] + hcc[q];
      L.tp_max = std::max(L.tp_max, hc[q]);
      L.tc_max = std::max(L.tc_max, hcc[q]);
    }
    MGFEM_HIP_TRY(hipMemcpyAsync(L.tp_off, ho.data(), ho.size() * sizeof(int), hipMemcpyHostToDevice, c->s));
    MGFEM_HIP_TRY(hipMemcpyAsync(L.tc_off, hco.data(), hco.size() * sizeof(int), hipMemcpyHostToDevice, c->s));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.tp_idx, std::max(1, ho[nt])));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.tp_coef, 9 * (size_t)std::max(1, ho[nt])));
    if (L.A32) MGFEM_HIP_TRY(ctx_alloc_t(c, &L.tp_coef32, 9 * (size_t)std::max(1, ho[nt])));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.tc_idx, std::max(1, hco[nt])));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.tc_pos, std::max(1, hco[nt])));
    if (nt > 0)
      hipLaunchKernelGGL(k_tile_plan, dim3(nt), dim3(256), 0, c->s, L.flags, L.A, L.A32, L.n, L.cutpos, L.N,
                         L.stride, L.bbox[0], L.bbox[2], L.bbox[1], L.bbox[3], TW, TH, ntx, L.tiles, 1, nullptr,
                         nullptr, L.tp_off, L.tc_off, L.tp_idx, L.tp_coef, L.tp_coef32, L.tc_idx, L.tc_pos);
    MGFEM_HIP_TRY(hipGetLastError());
    std::vector<int> meta(8 * (size_t)std::max(1, nt), 0);
    for (int q = 0; q < nt; ++q) {
      meta[8 * q + 0] = list[q];
      meta[8 * q + 1] = ho[q];
      meta[8 * q + 2] = hc[q];
      meta[8 * q + 3] = hco[q];
      meta[8 * q + 4] = hcc[q];
    }
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.tmeta, meta.size()));
    MGFEM_HIP_TRY(hipMemcpyAsync(L.tmeta, meta.data(), meta.size() * sizeof(int), hipMemcpyHostToDevice, c->s));
    // the host vectors must outlive the asynchronous copies
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
    // residual-restriction tiles: coarse tiles (the shape launch_resrestrict
    // uses for this level) with an active coarse node
    Level& C = c->lv[l + 1];
    if (!C.empty()) {
      const int CW = L.N >= 1024 ? 32 : 16, CH = L.N >= 1024 ? 16 : 8;
      const int cnx = (C.bbox[1] - C.bbox[0] + CW) / CW, cny = (C.bbox[3] - C.bbox[2] + CH) / CH;
      int* cact = nullptr;
      MGFEM_HIP_TRY(ctx_alloc_t(c, &cact, cnx * cny));
      hipLaunchKernelGGL(k_tile_active, dim3(cnx * cny), dim3(256), 0, c->s, C.flags, C.stride, C.bbox[0], C.bbox[2],
                         C.bbox[1], C.bbox[3], CW, CH, cnx, cny, cact);
      std::vector<int> hca(cnx * cny);
      MGFEM_HIP_TRY(hipMemcpyAsync(hca.data(), cact, hca.size() * sizeof(int), hipMemcpyDeviceToHost, c->s));
      MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
      std::vector<int> rl;
      for (int q = 0; q < cnx * cny; ++q)
        if (hca[q]) rl.push_back(q);
      MGFEM_HIP_TRY(ctx_alloc_t(c, &L.rr_tiles, std::max<size_t>(1, rl.size())));
      if (!rl.empty())
        MGFEM_HIP_TRY(hipMemcpyAsync(L.rr_tiles, rl.data(), rl.size() * sizeof(int), hipMemcpyHostToDevice, c->s));
      MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
      L.rr_ntiles = (int)rl.size();
    }
  }
  MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  return MGFEM_OK;
}

namespace {

// column setup of an extended coarse map: b of column j is the unit vector
// of the j0 + j-th active node (columns of nL values each)
__global__ void k_unit_cols(double* __restrict__ b, int64_t nL, const int* __restrict__ idx, int j0, int J) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < J) b[j * nL + idx[j0 + j]] = 1.0;
}

// B[i ld + j0 + j] = x_j[idx[i]]: row i of the map, columns j0 ... j0 + J - 1
__global__ void k_gather_cols(const double* __restrict__ x, int64_t nL, const int* __restrict__ idx, int n, int j0,
                              int J, double* __restrict__ B, int ld) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && j < J) B[(int64_t)i * ld + j0 + j] = x[(int64_t)j * nL + idx[i]];
}

// BT = B^T for n x n matrices with row stride ld, through 32 x 32 LDS tiles
__global__ __launch_bounds__(256) void k_transpose(const double* __restrict__ B, double* __restrict__ BT, int n,
                                                   int ld) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int r = threadIdx.x / 32; r < 32; r += 8) {
    const int i = by + r, j = bx + threadIdx.x % 32;
    tile[r][threadIdx.x % 32] = (i < n && j < n) ? B[(int64_t)i * ld + j] : 0.0;
  }
  __syncthreads();
  for (int r = threadIdx.x / 32; r < 32; r += 8) {
    const int i = bx + r, j = by + threadIdx.x % 32;
    if (i < n && j < n) BT[(int64_t)i * ld + j] = tile[threadIdx.x % 32][r];
  }
}

__global__ void k_zero_f64(double* __restrict__ p, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0.0;
}

// the multi-problem kernels in float64, the columns of a map as the problems
void col_launch(hipStream_t s, int kind, const void* tab, const int2* work, int nwork, int par, int prolong,
                int lds) {
  if (nwork <= 0) return;
  const unsigned grid = 8u * (unsigned)((nwork + 7) / 8);
  switch (kind) {
    case kTeamSweep:
      hipLaunchKernelGGL((k_sweep_multi<double, 16, 16, 512>), dim3(grid), dim3(512), 0, s,
                         static_cast<const SweepEntry<double>*>(tab), work, nwork, par, 0, prolong);
      break;
    case kTeamCut:
      hipLaunchKernelGGL(k_cut_multi<double>, dim3(grid), dim3(kCutThreads), lds, s,
                         static_cast<const CutEntry<double>*>(tab), work, nwork, par);
      break;
    case kTeamRR:
      hipLaunchKernelGGL((k_resrestrict_multi<double, 16, 8, 512>), dim3(grid), dim3(512), 0, s,
                         static_cast<const RrEntry<double>*>(tab), work, nwork, par, 0);
      break;
    case kTeamMap:
      hipLaunchKernelGGL(k_coarse_apply_multi<double>, dim3(nwork), dim3(64 * kMapWaves), lds, s,
                         static_cast<const MapEntry<double>*>(tab), work, nwork);
      break;
  }
}

template <class E>
int upload_table(mgfem_ctx* c, const std::vector<E>& h, void** dev) {
  MGFEM_HIP_TRY(hipMalloc(dev, h.size() * sizeof(E)));
  MGFEM_HIP_TRY(hipMemcpyAsync(*dev, h.data(), h.size() * sizeof(E), hipMemcpyHostToDevice, c->s));
  return MGFEM_OK;
}

}  // namespace

// Extend the coarse map one level up, as long as that level is small: the
// V-cycle from zero on level L (its smoothing, residual and restriction, the
// coarse part through the map of level L + 1, prolongation and smoothing) is
// again a fixed linear map of level L's right-hand side.  Its columns are the
// results on the unit vectors, computed in batches of columns with the
// multi-problem kernels in float64 (every column is a problem of its own with
// its own vectors and the level's operators); the transposed cycle's map is
// its transpose (the transposed cycle is the cycle's adjoint).  Not for
// W-cycles (their coarse part repeats), nor up to level 1 of the two-grid
// scheme (its first coarse problem takes coarse_cycles cycles).
int extend_coarse_map(mgfem_ctx* c) {
  CoarseMap& M = c->cplan.map;
  const char* env = std::getenv("MGFEM_NO_MAP_EXTENSION");
  if (env && env[0] && env[0] != '0') return MGFEM_OK;
  while (M.level >= 2) {
    const int C = M.level, L = C - 1;
    if (!M.f64[0] || !M.f64[1] || M.reps != 1 || c->p.cycle == MGFEM_CYCLE_W || c->p.nu2 < 1) break;
    if (c->p.cycle == MGFEM_CYCLE_TWO_GRID && L < 2) break;
    Level& Ll = c->lv[L];
    Level& Lc = c->lv[C];
    if (Ll.empty() || Ll.n_active > kMaxMapNodes || sweep_shape(c, L) != kShapeSmall || Ll.N >= 1024) break;
    const bool has_cut = c->p.eta > 0 && Ll.cut_off[4] > 0;
    if (has_cut && !Ll.cp.ok) break;
    // the active nodes of level L, ascending: rows and columns of the new map
    std::vector<uint8_t> fl(Ll.n);
    MGFEM_HIP_TRY(hipMemcpyAsync(fl.data(), Ll.flags, Ll.n, hipMemcpyDeviceToHost, c->s));
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
    std::vector<int> idx;
    for (int64_t k = 0; k < Ll.n; ++k)
      if (fl[k] & kFlagActive) idx.push_back((int)k);
    const int n = (int)idx.size();
    if (n == 0 || n > kMaxMapNodes) break;
    const int ld = (n + 15) / 16 * 16;
    double* B = nullptr;
    int* didx = nullptr;
    MGFEM_HIP_TRY(ctx_alloc_t(c, &B, (size_t)ld * n));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &didx, n));
    MGFEM_HIP_TRY(hipMemcpyAsync(didx, idx.data(), n * sizeof(int), hipMemcpyHostToDevice, c->s));
    // vectors of a batch of J columns (freed below)
    const int J = std::min(n, 512);
    const int64_t nL = Ll.n, nC = Lc.n;
    const int64_t ncL = std::max(1, Ll.cut_off[4]), ncC = std::max(1, Lc.cut_off[4]);
    const int64_t total = 3 * J * nL + J * ncL + 3 * J * nC + J * ncC;
    double* buf = nullptr;
    MGFEM_HIP_TRY(hipMalloc(&buf, total * sizeof(double)));
    double* XL = buf;               // buffer 0 of column j at XL + j nL, buffer 1 at XL + (J + j) nL
    double* bL = XL + 2 * J * nL;
    double* sL = bL + J * nL;
    double* XC = sL + J * ncL;      // level C: buffer 0 (the map's output) and buffer 1
    double* bC = XC + 2 * J * nC;
    double* sC = bC + J * nC;
    std::vector<SweepEntry<double>> ts(J);
    std::vector<CutEntry<double>> tc(J);
    std::vector<RrEntry<double>> tr(J);
    std::vector<MapEntry<double>> tm(J);
    for (int j = 0; j < J; ++j) {
      SweepEntry<double>& e = ts[j];
      e.a = sweep_args<double, 16, 16>(c, L, false, false, false);
      e.a.b = bL + j * nL;
      e.a.snap = sL + j * ncL;
      e.a.sc = Lc.stride;
      e.X[0] = XL + j * nL;
      e.X[1] = XL + (J + j) * nL;
      e.XC[0] = XC + j * nC;
      e.XC[1] = XC + (J + j) * nC;
      e.xc_fixed = 1;
      if (has_cut) {
        CutEntry<double>& u = tc[j];
        u.a = cut_args<double>(c, L, false);
        u.a.b = bL + j * nL;
        u.a.snap = sL + j * ncL;
        u.X[0] = e.X[0];
        u.X[1] = e.X[1];
      }
      RrEntry<double>& r = tr[j];
      r.a = rr_args<double, 16, 8>(c, L);
      r.a.b = bL + j * nL;
      r.a.bc = bC + j * nC;
      r.a.snapc = sC + j * ncC;
      r.X[0] = e.X[0];
      r.X[1] = e.X[1];
      r.XC[0] = XC + j * nC;
      r.XC[1] = XC + (J + j) * nC;
      r.xc_fixed = 1;
      MapEntry<double>& m = tm[j];
      m.B = M.f64[0];
      m.ld = M.ld;
      m.idx = M.idx;
      m.n = M.n;
      m.b = bC + j * nC;
      m.x = XC + j * nC;
    }
    void *dts = nullptr, *dtc = nullptr, *dtr = nullptr, *dtm = nullptr;
    int rc = upload_table(c, ts, &dts);
    if (!rc) rc = upload_table(c, tc, &dtc);
    if (!rc) rc = upload_table(c, tr, &dtr);
    if (!rc) rc = upload_table(c, tm, &dtm);
    // work lists, column by column (the first Jc columns are a prefix)
    const int us = Ll.ntiles, uc = has_cut ? Ll.cp.ngroups : 0, ur = Lc.empty() ? 0 : Ll.rr_ntiles;
    const int um = (M.n + kMapWaves - 1) / kMapWaves;
    std::vector<int2> w;
    for (int j = 0; j < J; ++j)
      for (int q = 0; q < us; ++q) w.push_back(make_int2(j, q));
    for (int j = 0; j < J; ++j)
      for (int q = 0; q < uc; ++q) w.push_back(make_int2(j, q));
    for (int j = 0; j < J; ++j)
      for (int q = 0; q < ur; ++q) w.push_back(make_int2(j, q));
    for (int j = 0; j < J; ++j)
      for (int q = 0; q < um; ++q) w.push_back(make_int2(j, q));
    int2* dw = nullptr;
    if (!rc && hipMalloc(&dw, w.size() * sizeof(int2)) != hipSuccess) rc = MGFEM_ERR_OOM;
    if (!rc && hipMemcpyAsync(dw, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice, c->s) != hipSuccess)
      rc = MGFEM_ERR_HIP;
    const int2* ws = dw;
    const int2* wc = dw + (size_t)J * us;
    const int2* wr = wc + (size_t)J * uc;
    const int2* wm = wr + (size_t)J * ur;
    const int cut_lds = Ll.cp.lds64, map_lds = M.ld * (int)sizeof(double);
    for (int j0 = 0; j0 < n && !rc; j0 += J) {
      const int Jc = std::min(J, n - j0);
      hipLaunchKernelGGL(k_zero_f64, dim3(nblk(total, 256)), dim3(256), 0, c->s, buf, total);
      hipLaunchKernelGGL(k_unit_cols, dim3(nblk(Jc, 256)), dim3(256), 0, c->s, bL, nL, (const int*)didx, j0, Jc);
      int par = 0;
      auto smooth_cols = [&](bool prolong) {
        col_launch(c->s, kTeamSweep, dts, ws, Jc * us, par, prolong ? 1 : 0, 0);
        par ^= 1;
        if (has_cut) col_launch(c->s, kTeamCut, dtc, wc, Jc * uc, par, 0, cut_lds);
      };
      for (int st = 0; st < c->p.nu1; ++st) smooth_cols(false);
      col_launch(c->s, kTeamRR, dtr, wr, Jc * ur, par, 0, 0);
      col_launch(c->s, kTeamMap, dtm, wm, Jc * um, 0, 0, map_lds);
      smooth_cols(true);  // x + P x_c, then the step
      for (int st = 1; st < c->p.nu2; ++st) smooth_cols(false);
      hipLaunchKernelGGL(k_gather_cols, dim3(nblk(Jc, 256), n), dim3(256), 0, c->s,
                         (const double*)(XL + (par ? J * nL : 0)), nL, (const int*)didx, n, j0, Jc, B, ld);
      if (hipGetLastError() != hipSuccess) rc = MGFEM_ERR_HIP;
    }
    if (hipStreamSynchronize(c->s) != hipSuccess && !rc) rc = MGFEM_ERR_HIP;
    (void)hipFree(dw);
    (void)hipFree(dts);
    (void)hipFree(dtc);
    (void)hipFree(dtr);
    (void)hipFree(dtm);
    (void)hipFree(buf);
    if (rc) {
      c->last_error = "coarse map extension to level " + std::to_string(L) + " failed";
      return rc;
    }
    double* BT = nullptr;
    MGFEM_HIP_TRY(ctx_alloc_t(c, &BT, (size_t)ld * n));
    hipLaunchKernelGGL(k_transpose, dim3((n + 31) / 32, (n + 31) / 32), dim3(256), 0, c->s, (const double*)B, BT, n,
                       ld);
    float* B32 = nullptr;
    if (c->p.precision == MGFEM_PREC_MIXED) {
      MGFEM_HIP_TRY(ctx_alloc_t(c, &B32, (size_t)ld * n));
      hipLaunchKernelGGL(k_f64_to_f32, dim3(nblk((int64_t)ld * n, 256)), dim3(256), 0, c->s, (const double*)B, B32,
                         (int64_t)ld * n);
    }
    MGFEM_HIP_TRY(hipGetLastError());
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
    M.level = L;
    M.n = n;
    M.ld = ld;
    M.idx = didx;
    M.f64[0] = B;
    M.f64[1] = BT;
    M.f32 = B32;
  }
  return MGFEM_OK;
}

int build_coarse_map(mgfem_ctx* c, bool forward_only) {
  CoarsePlan& P = c->cplan;
  CoarseMap& M = P.map;
  if (P.lc < 0 || M.n <= 0 || M.n > kMaxMapNodes) return MGFEM_OK;
  {
    const char* env = std::getenv("MGFEM_NO_COARSE_MAP");
    if (env && env[0] && env[0] != '0') return MGFEM_OK;
  }
  // the cycles one coarse-part launch runs: gamma* (the two-grid scheme solves
  // its first coarse problem with coarse_cycles cycles when that problem is
  // the first level of the coarse part)
  const bool two_grid = c->p.cycle == MGFEM_CYCLE_TWO_GRID && P.lc == 1;
  M.reps = two_grid ? c->p.coarse_cycles : (c->p.cycle == MGFEM_CYCLE_W ? 2 : 1);
  M.level = P.lc;
  M.ld = (M.n + 15) / 16 * 16;
  const size_t cnt = (size_t)M.ld * M.n;
  for (int rev = 0; rev < (forward_only ? 1 : 2); ++rev) {
    MGFEM_HIP_TRY(ctx_alloc_t(c, &M.f64[rev], cnt));  // zeroed: the padding columns stay 0
    CoarseArgs<double> a = coarse_args<double>(c, rev != 0, M.reps);
    a.unit = 1;
    a.map_out = M.f64[rev];
    a.map_ld = M.ld;
    hipLaunchKernelGGL(k_coarse<double>, dim3(M.n), dim3(kCoarseThreads), P.lds64, c->s, a);
    MGFEM_HIP_TRY(hipGetLastError());
  }
  if (c->p.precision == MGFEM_PREC_MIXED) {
    MGFEM_HIP_TRY(ctx_alloc_t(c, &M.f32, cnt));
    hipLaunchKernelGGL(k_f64_to_f32, dim3(nblk((int64_t)cnt, 256)), dim3(256), 0, c->s,
                       (const double*)M.f64[0], M.f32, (int64_t)cnt);
    MGFEM_HIP_TRY(hipGetLastError());
  }
  MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  if (!forward_only) return extend_coarse_map(c);
  return MGFEM_OK;
}

void smooth_level(mgfem_ctx* c, int l, bool reverse, bool fp32) {
  if (fp32) smooth<float>(c, l, reverse);
  else smooth<double>(c, l, reverse);
}

void set_kernel_attributes() {
  // dynamic LDS beyond the default limit for the two LDS-resident kernels
  int dev = 0, lds = 65536;
  if (hipGetDevice(&dev) != hipSuccess) return;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_cut<double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_cut<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_cut_multi<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_cut_multi<double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_coarse<double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_coarse<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipGetLastError();
}

void gather_snap(mgfem_ctx* c, int l, bool fp32) {
  Level& L = c->lv[l];
  const int cnt = L.cut_off[4];
  if (cnt == 0) return;
  if (fp32)
    hipLaunchKernelGGL(k_snap_gather<float>, dim3(nblk(cnt, 256)), dim3(256), 0, c->s, L.cut_list, cnt,
                       (const float*)L.X32[L.cur], L.snap32);
  else
    hipLaunchKernelGGL(k_snap_gather<double>, dim3(nblk(cnt, 256)), dim3(256), 0, c->s, L.cut_list, cnt,
                       (const double*)L.X[L.cur], L.snap);
}

}  // namespace mgfem

// ===========================================================================
// Batched solves in one persistent launch.
//
// Every workgroup (1024 threads) takes whole problems from a work queue (an
// atomic counter over the problems ordered by decreasing size) and solves
// each one alone: no workgroup ever waits for another, and each exits when
// the queue is empty.  Per problem: F = M f + G g, then float64 defect
// correction around float32 V(nu1, nu2) cycles.  On the grid levels above the
// LDS-resident coarse part, a colour phase updates its nodes in place in
// global memory (one workgroup, so a barrier separates the phases; nodes of
// one colour never neighbour each other); the coarse levels run in LDS as in
// the single-problem solver.  Threads cover each colour sub-lattice in
// footprints of tx x (1024 / tx) nodes; tx is chosen by the autotuner.
// ===========================================================================
namespace mgfem {
namespace {

template <class F>
__device__ inline void wg_for_sublattice(int i0, int i1, int j0, int j1, int cx, int cy, int tx, F&& f) {
  // nodes (i, j) of the box with i = cx, j = cy (mod 2); cx = -1 / cy = -1: every node
  const int fi = cx < 0 ? i0 : i0 + ((cx - i0) & 1), fj = cy < 0 ? j0 : j0 + ((cy - j0) & 1);
  const int di = cx < 0 ? 1 : 2, dj = cy < 0 ? 1 : 2;
  if (fi > i1 || fj > j1) return;
  const int ni = (i1 - fi) / di + 1, nj = (j1 - fj) / dj + 1;
  const int ty = 1024 / tx;
  const int lx = threadIdx.x % tx, ly = threadIdx.x / tx;
  for (int pj = 0; pj < nj; pj += ty) {
    const int tj = pj + ly;
    if (tj >= nj) continue;
    for (int pi = 0; pi < ni; pi += tx) {
      const int ti = pi + lx;
      if (ti < ni) f(fi + di * ti, fj + dj * tj);
    }
  }
}

// row product of node k (i, j) against x in global memory; returns the full
// product, with the diagonal and the off-diagonal part; rows on the grid edge
// skip the neighbours outside the grid
template <class T>
__device__ inline T glob_row(const T* __restrict__ A, int64_t n, const T* x, int64_t k, int i, int j, int N, int s,
                             bool stored, T& diag, T& off) {
  if (stored) {
    diag = A[4 * n + k];
    if (i > 0 && j > 0 && i < N && j < N) {
      off = A[k] * x[k - s - 1] + A[n + k] * x[k - s] + A[2 * n + k] * x[k - s + 1] + A[3 * n + k] * x[k - 1] +
            A[5 * n + k] * x[k + 1] + A[6 * n + k] * x[k + s - 1] + A[7 * n + k] * x[k + s] +
            A[8 * n + k] * x[k + s + 1];
    } else {
      off = T(0);
      for (int q = 0; q < 9; ++q) {
        if (q == 4) continue;
        const int ii = i + q % 3 - 1, jj = j + q / 3 - 1;
        if (ii < 0 || jj < 0 || ii > N || jj > N) continue;
        off += A[q * n + k] * x[ii + (int64_t)jj * s];
      }
    }
  } else {  // interior Q1 row: every neighbour exists
    diag = T(8) / T(3);
    off = -((x[k - s - 1] + x[k - s] + x[k - s + 1]) + (x[k - 1] + x[k + 1]) +
            (x[k + s - 1] + x[k + s] + x[k + s + 1])) * T(1.0 / 3.0);
  }
  return diag * x[k] + off;
}

struct BLevel {
  int N, s, i0, i1, j0, j1;
  int64_t n;
  const float* A;
  const uint8_t* fl;
  float* x;
  float* r;
  float* b;
  const int* cut;
  int cut_off[5];
};

constexpr int kMaxBLevels = 16;

struct BProb {
  int nlev;  // grid levels above the coarse workgroup part
  int N0, s0, i0, i1, j0, j1;
  int64_t n0;
  const double* A64;
  const uint8_t* fl0;
  const double* M;
  const double* G;
  double* F;
  double* r64;
  BLevel lev[kMaxBLevels];
  CoarseArgs<float> ca;
};

struct BatchArgs {
  const BProb* probs;
  const int* order;
  int count;
  const double* const* f;
  const double* const* g;
  double* const* u;
  double* hist;  // count x (max_cycles + 1)
  int* ncyc;
  double tol;
  int max_cycles, nu1, nu2, eta, tx;
  int inner;  // float32 cycles per float64 step
  unsigned int* queue;
};

// workgroup reduction of (max, sum); every thread gets the result
__device__ inline void wg_reduce2(double& mx, double& sm, double* red) {
  for (int o = 32; o > 0; o >>= 1) {
    mx = nanmax2(mx, __shfl_xor(mx, o));
    sm += __shfl_xor(sm, o);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = mx;
    red[2 * w + 1] = sm;
  }
  __syncthreads();
  mx = 0.0;
  sm = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
    mx = nanmax2(mx, red[2 * q]);
    sm += red[2 * q + 1];
  }
  __syncthreads();
}

__device__ void b_smooth(const BLevel& L, int eta, int tx) {
  for (int c = 0; c < 4; ++c) {
    wg_for_sublattice(L.i0, L.i1, L.j0, L.j1, c & 1, c >> 1, tx, [&](int i, int j) {
      const int64_t k = i + (int64_t)j * L.s;
      const uint8_t f = L.fl[k];
      if (!(f & kFlagActive)) return;
      float diag, off;
      (void)glob_row<float>(L.A, L.n, L.x, k, i, j, L.N, L.s, (f & kFlagStored) != 0, diag, off);
      L.x[k] = (L.b[k] - off) / diag;
    });
    __syncthreads();
  }
  for (int e = 0; e < eta; ++e)
    for (int c = 0; c < 4; ++c) {
      for (int t = L.cut_off[c] + threadIdx.x; t < L.cut_off[c + 1]; t += blockDim.x) {
        const int64_t k = L.cut[t];
        float diag, off;
        (void)glob_row<float>(L.A, L.n, L.x, k, (int)(k % L.s), (int)(k / L.s), L.N, L.s, true, diag, off);
        L.x[k] = (L.b[k] - off) / diag;
      }
      __syncthreads();
    }
}

__device__ void b_restrict(const BLevel& L, const BLevel& C, int tx) {
  wg_for_sublattice(L.i0, L.i1, L.j0, L.j1, -1, -1, tx, [&](int i, int j) {
    const int64_t k = i + (int64_t)j * L.s;
    const uint8_t f = L.fl[k];
    if (!(f & kFlagActive)) return;
    float diag, off;
    L.r[k] = L.b[k] - glob_row<float>(L.A, L.n, L.x, k, i, j, L.N, L.s, (f & kFlagStored) != 0, diag, off);
  });
  __syncthreads();
  wg_for_sublattice(C.i0, C.i1, C.j0, C.j1, -1, -1, tx, [&](int I, int J) {
    const int64_t kc = I + (int64_t)J * C.s;
    if (!(C.fl[kc] & kFlagActive)) return;
    const int fi = 2 * I, fj = 2 * J;
    float v = 0.f;
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = fj + dj;
      if (jj < 0 || jj > L.N) continue;
      const float* rr = L.r + (int64_t)jj * L.s;
      float row = rr[fi], side = 0.f;
      if (fi > 0) side += rr[fi - 1];
      if (fi < L.N) side += rr[fi + 1];
      v += (dj == 0 ? 1.f : 0.5f) * (row + 0.5f * side);
    }
    C.b[kc] = v;
    C.x[kc] = 0.f;
  });
  __syncthreads();
}

__device__ void b_prolong(const BLevel& L, const BLevel& C, int tx) {
  wg_for_sublattice(L.i0, L.i1, L.j0, L.j1, -1, -1, tx, [&](int i, int j) {
    const int64_t k = i + (int64_t)j * L.s;
    if (!(L.fl[k] & kFlagActive)) return;
    const int I0 = i >> 1, I1 = (i + 1) >> 1, J0 = j >> 1, J1 = (j + 1) >> 1;
    const float* xc = C.x;
    const int64_t r0 = (int64_t)J0 * C.s, r1 = (int64_t)J1 * C.s;
    L.x[k] += 0.25f * ((xc[I0 + r0] + xc[I1 + r0]) + (xc[I0 + r1] + xc[I1 + r1]));
  });
  __syncthreads();
}

// float64 residual r64 = F - A u over level 0 with (max |r|, sum r^2)
__device__ void b_residual64(const BProb& P, const double* u, double& mx, double& sm, int tx, double* red) {
  mx = 0.0;
  sm = 0.0;
  wg_for_sublattice(P.i0, P.i1, P.j0, P.j1, -1, -1, tx, [&](int i, int j) {
    const int64_t k = i + (int64_t)j * P.s0;
    const uint8_t f = P.fl0[k];
    if (!(f & kFlagActive)) return;
    double diag, off;
    const double r =
        P.F[k] - glob_row<double>(P.A64, P.n0, u, k, i, j, P.N0, P.s0, (f & kFlagStored) != 0, diag, off);
    P.r64[k] = r;
    mx = nanmax2(mx, fabs(r));
    sm += r * r;
  });
  wg_reduce2(mx, sm, red);
}

__device__ void solve_one(const BatchArgs& a, int p, unsigned char* base, int* sdesc, double* red) {
  const BProb& P = a.probs[p];
  double* u = a.u[p];
  const double* f = a.f[p];
  const double* g = a.g[p];
  const int tx = a.tx;
  double* hist = a.hist + (int64_t)p * (a.max_cycles + 1);
  // u = 0 everywhere; F = M f + G g on the active nodes
  for (int64_t k = threadIdx.x; k < P.n0; k += blockDim.x) u[k] = 0.0;
  wg_for_sublattice(P.i0, P.i1, P.j0, P.j1, -1, -1, tx, [&](int i, int j) {
    const int64_t k = i + (int64_t)j * P.s0;
    double acc = 0.0;
    if (P.fl0[k] & kFlagActive)
      for (int q = 0; q < 9; ++q) {
        const int ii = i + q % 3 - 1, jj = j + q / 3 - 1;
        if (ii < 0 || jj < 0 || ii > P.N0 || jj > P.N0) continue;
        const int64_t kk = ii + (int64_t)jj * P.s0;
        const double m = P.M[q * P.n0 + k], gg = P.G[q * P.n0 + k];
        if (m != 0.0) acc += m * f[kk];
        if (gg != 0.0) acc += gg * g[kk];
      }
    P.F[k] = acc;
  });
  __syncthreads();
  double mx, sm;
  b_residual64(P, u, mx, sm, tx, red);
  hist[0] = mx;
  const double fnorm = mx;
  int m = 0;
  double prev = mx;
  int grow = 0;
  // rel_tol <= 0: exactly max_cycles cycles
  while (m < a.max_cycles && !(a.tol > 0.0 && mx <= a.tol * fnorm) && mx == mx) {
    // inner float32 cycles on A e = r, the first from e = 0
    const BLevel& L0 = P.lev[0];
    wg_for_sublattice(P.i0, P.i1, P.j0, P.j1, -1, -1, tx, [&](int i, int j) {
      const int64_t k = i + (int64_t)j * P.s0;
      L0.b[k] = (float)P.r64[k];
      L0.x[k] = 0.f;
    });
    __syncthreads();
    for (int ic = 0; ic < a.inner; ++ic) {
      for (int l = 0; l < P.nlev; ++l) {
        for (int s = 0; s < a.nu1; ++s) b_smooth(P.lev[l], a.eta, tx);
        b_restrict(P.lev[l], P.lev[l + 1], tx);
      }
      coarse_body<float>(P.ca, base, sdesc);
      for (int l = P.nlev - 1; l >= 0; --l) {
        b_prolong(P.lev[l], P.lev[l + 1], tx);
        for (int s = 0; s < a.nu2; ++s) b_smooth(P.lev[l], a.eta, tx);
      }
    }
    // float64 update and residual
    wg_for_sublattice(P.i0, P.i1, P.j0, P.j1, -1, -1, tx, [&](int i, int j) {
      const int64_t k = i + (int64_t)j * P.s0;
      if (P.fl0[k] & kFlagActive) u[k] += (double)L0.x[k];
    });
    __syncthreads();
    b_residual64(P, u, mx, sm, tx, red);
    ++m;
    hist[m] = mx;
    grow = mx > prev ? grow + 1 : 0;
    if (grow >= 3) break;
    prev = mx;
  }
  if (threadIdx.x == 0) a.ncyc[p] = m;
  __syncthreads();
}

__global__ __launch_bounds__(1024) void k_batched(BatchArgs a) {
  extern __shared__ __align__(16) unsigned char base[];
  __shared__ int sdesc[kDesc * kMaxWgLevels];
  __shared__ double red[32];
  __shared__ int sidx;
  while (true) {
    if (threadIdx.x == 0) sidx = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    const int q = sidx;
    __syncthreads();
    if (q >= a.count) break;  // queue empty: every workgroup ends here
    solve_one(a, a.order[q], base, sdesc, red);
  }
}

}  // namespace

}  // namespace mgfem

namespace mgfem {

size_t bprob_size() { return sizeof(BProb); }

// one BProb per member context (set up in mixed precision)
void build_batch_layout(std::vector<mgfem_ctx*>& members, std::vector<unsigned char>& probs_bytes, int& lds) {
  probs_bytes.assign(members.size() * sizeof(BProb), 0);
  lds = 0;
  for (size_t i = 0; i < members.size(); ++i) {
    mgfem_ctx* c = members[i];
    BProb P{};
    const int lc = c->cplan.lc;
    P.nlev = lc;
    Level& L0 = c->lv[0];
    P.N0 = L0.N;
    P.s0 = L0.stride;
    P.n0 = L0.n;
    P.i0 = L0.bbox[0];
    P.i1 = L0.bbox[1];
    P.j0 = L0.bbox[2];
    P.j1 = L0.bbox[3];
    P.A64 = L0.A;
    P.fl0 = L0.flags;
    P.M = c->M;
    P.G = c->G;
    P.F = c->F;
    P.r64 = c->F64tmp;
    for (int l = 0; l <= lc && l < kMaxBLevels; ++l) {
      Level& L = c->lv[l];
      BLevel& B = P.lev[l];
      B.N = L.N;
      B.s = L.stride;
      B.n = L.n;
      B.i0 = L.bbox[0];
      B.i1 = L.bbox[1];
      B.j0 = L.bbox[2];
      B.j1 = L.bbox[3];
      B.A = L.A32;
      B.fl = L.flags;
      B.x = L.X32[0];
      B.r = L.X32[1];
      B.b = L.b32;
      B.cut = L.cut_list;
      for (int q = 0; q < 5; ++q) B.cut_off[q] = L.cut_off[q];
    }
    CoarsePlan& CP = c->cplan;
    CoarseArgs<float>& A = P.ca;
    A.desc = CP.desc + kDesc * CP.ndesc;
    A.coef = CP.coef32;
    A.slot = CP.slot;
    A.cutl = CP.cutl;
    A.actl = CP.actl;
    A.inv = CP.inv;
    A.cidx = nullptr;
    A.img = CP.img32;
    A.img_bytes = CP.static32;
    A.lds_bytes = CP.lds32;
    A.cn = c->coarse_n;
    A.nlev = CP.ndesc;
    A.b_top = c->lv[lc].b32;
    A.x_top = c->lv[lc].X32[0];
    A.s_top = c->lv[lc].stride;
    A.nu1 = c->p.nu1;
    A.nu2 = c->p.nu2;
    A.eta = c->p.eta;
    A.reverse = 0;
    A.gstar = 1;
    A.reps = 1;
    lds = std::max(lds, CP.lds32);
    std::memcpy(probs_bytes.data() + i * sizeof(BProb), &P, sizeof(BProb));
  }
}

float launch_batched(mgfem_ctx* b, BatchDevice& d, int count, double tol, int max_cycles, int tx) {
  BatchArgs a;
  a.probs = reinterpret_cast<const BProb*>(d.probs);
  a.order = d.order;
  a.count = count;
  a.f = d.f;
  a.g = d.g;
  a.u = d.u;
  a.hist = d.hist;
  a.ncyc = d.ncyc;
  a.tol = tol;
  a.max_cycles = max_cycles;
  a.nu1 = b->p.nu1;
  a.nu2 = b->p.nu2;
  a.eta = b->p.eta;
  a.tx = tx;
  a.inner = b->p.inner_cycles;
  a.queue = d.queue;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_batched), hipFuncAttributeMaxDynamicSharedMemorySize,
                            d.lds);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipMemsetAsync(d.queue, 0, sizeof(unsigned int), b->s);
  (void)hipEventRecord(e0, b->s);
  hipLaunchKernelGGL(k_batched, dim3(std::min(count, cus)), dim3(1024), d.lds, b->s, a);
  (void)hipEventRecord(e1, b->s);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

}  // namespace mgfem
