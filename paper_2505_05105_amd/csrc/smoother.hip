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
//  k_coarse     the V-cycle of all remaining coarse levels in one workgroup.
#include <algorithm>
#include <cmath>

#include "mgfem_internal.h"

namespace mgfem {
namespace {

constexpr int kHalo = 4;

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
  int reverse;
};

// product of the stored stencil row at node k with LDS values around q
template <class T, int RW>
__device__ inline T stored_row(const T* __restrict__ A, int64_t n, int64_t k, const T* su, int q, T& diag) {
  diag = A[4 * n + k];
  T acc = diag * su[q];
  acc += A[k] * su[q - RW - 1];
  acc += A[n + k] * su[q - RW];
  acc += A[2 * n + k] * su[q - RW + 1];
  acc += A[3 * n + k] * su[q - 1];
  acc += A[5 * n + k] * su[q + 1];
  acc += A[6 * n + k] * su[q + RW - 1];
  acc += A[7 * n + k] * su[q + RW];
  acc += A[8 * n + k] * su[q + RW + 1];
  return acc;
}

template <class T, int RW>
__device__ inline T q1_row(const T* su, int q, T& diag) {
  diag = T(8) / T(3);
  const T nb = (su[q - RW - 1] + su[q - RW] + su[q - RW + 1]) + (su[q - 1] + su[q + 1]) +
               (su[q + RW - 1] + su[q + RW] + su[q + RW + 1]);
  return diag * su[q] - nb / T(3);
}

template <class T, int TW, int TH>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs<T> a) {
  constexpr int RW = TW + 2 * kHalo, RH = TH + 2 * kHalo;
  constexpr int BW = RW - 2, BH = RH - 2;
  __shared__ T su[RH * RW];
  __shared__ T sb[BH * BW];
  __shared__ uint8_t sf[BH * BW];
  const int xcd = blockIdx.x & 7, loc = blockIdx.x >> 3;
  const int t = xcd * a.per + loc;
  if (t >= a.ntx * a.nty) return;  // uniform for the whole block, before any barrier
  const int tx = t % a.ntx, ty = t / a.ntx;
  const int ox = a.i0 + tx * TW - kHalo, oy = a.j0 + ty * TH - kHalo;
  for (int q = threadIdx.x; q < RW * RH; q += blockDim.x) {
    const int gi = ox + q % RW, gj = oy + q / RW;
    su[q] = (gi >= 0 && gj >= 0 && gi <= a.N && gj <= a.N) ? a.xin[gi + (int64_t)gj * a.s] : T(0);
  }
  for (int q = threadIdx.x; q < BW * BH; q += blockDim.x) {
    const int gi = ox + 1 + q % BW, gj = oy + 1 + q / BW;
    uint8_t f = 0;
    T bv = T(0);
    if (gi >= 0 && gj >= 0 && gi <= a.N && gj <= a.N) {
      const int64_t k = gi + (int64_t)gj * a.s;
      f = a.fl[k];
      if (f & kFlagActive) bv = a.b[k];
    }
    sf[q] = f;
    sb[q] = bv;
  }
  __syncthreads();
  for (int p = 0; p < 4; ++p) {
    const int c = a.reverse ? 3 - p : p;
    const int cx = c & 1, cy = c >> 1;
    const int lo = p + 1;
    const int fx = lo + ((cx - (ox + lo)) & 1), fy = lo + ((cy - (oy + lo)) & 1);
    const int nx = (RW - 1 - p - fx + 1) / 2, ny = (RH - 1 - p - fy + 1) / 2;
    for (int q = threadIdx.x; q < nx * ny; q += blockDim.x) {
      const int ri = fx + 2 * (q % nx), rj = fy + 2 * (q / nx);
      const int bq = (ri - 1) + (rj - 1) * BW;
      const uint8_t f = sf[bq];
      if (!(f & kFlagActive)) continue;
      const int sq = ri + rj * RW;
      T diag, ax;
      if (f & kFlagStored) {
        const int64_t k = (ox + ri) + (int64_t)(oy + rj) * a.s;
        ax = stored_row<T, RW>(a.A, a.n, k, su, sq, diag);
      } else {
        ax = q1_row<T, RW>(su, sq, diag);
      }
      su[sq] += (sb[bq] - ax) / diag;
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < TW * TH; q += blockDim.x) {
    const int ri = kHalo + q % TW, rj = kHalo + q / TW;
    const int gi = ox + ri, gj = oy + rj;
    if (gi > a.i1 || gj > a.j1) continue;
    const uint8_t f = sf[(ri - 1) + (rj - 1) * BW];
    if (!(f & kFlagActive)) continue;
    const int64_t k = gi + (int64_t)gj * a.s;
    const T v = su[ri + rj * RW];
    a.xout[k] = v;
    if (f & kFlagCut) a.snap[a.cutpos[k]] = v;
  }
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
  T* x;
  const T* b;
  const T* A;
  const T* snap;
  int64_t n;
  int eta, reverse;
};

__constant__ int kNbrPlane[8] = {0, 1, 2, 3, 5, 6, 7, 8};

template <class T>
__global__ __launch_bounds__(256) void k_cut(CutArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int* gi = a.g_info + 9 * blockIdx.x;
  const int cl_off = gi[0], cl_cnt = gi[1], ext_off = gi[2], ext_cnt = gi[3];
  T* sval = reinterpret_cast<T*>(smem);
  T* sbv = sval + cl_cnt;
  T* scoef = sbv + cl_cnt;
  T* sext = scoef + 9 * cl_cnt;
  int16_t* snbr = reinterpret_cast<int16_t*>(sext + ext_cnt);
  for (int t = threadIdx.x; t < cl_cnt; t += blockDim.x) {
    const int64_t k = a.cl_node[cl_off + t];
    sval[t] = a.snap[a.cl_q[cl_off + t]];
    sbv[t] = a.b[k];
    for (int p = 0; p < 9; ++p) scoef[9 * t + p] = a.A[p * a.n + k];
    for (int e = 0; e < 8; ++e) snbr[8 * t + e] = a.cl_nbr[8 * (int64_t)(cl_off + t) + e];
  }
  for (int t = threadIdx.x; t < ext_cnt; t += blockDim.x) {
    const int src = a.ext_src[ext_off + t];
    sext[t] = src >= 0 ? a.x[src] : a.snap[-(1 + src)];
  }
  __syncthreads();
  for (int sweep = 0; sweep < a.eta; ++sweep) {
    for (int p = 0; p < 4; ++p) {
      const int c = a.reverse ? 3 - p : p;
      const int lo = gi[4 + c], hi = gi[5 + c];
      for (int t = lo + threadIdx.x; t < hi; t += blockDim.x) {
        const T diag = scoef[9 * t + 4];
        T acc = sbv[t] - diag * sval[t];
        for (int e = 0; e < 8; ++e) {
          const int r = snbr[8 * t + e];
          if (r < 0) continue;
          const T v = r < cl_cnt ? sval[r] : sext[r - cl_cnt];
          acc -= scoef[9 * t + kNbrPlane[e]] * v;
        }
        sval[t] += acc / diag;
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < cl_cnt; t += blockDim.x)
    if (a.cl_own[cl_off + t]) a.x[a.cl_node[cl_off + t]] = sval[t];
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
};

template <class T, int CW, int CH>
__global__ __launch_bounds__(256) void k_resrestrict(ResArgs<T> a) {
  constexpr int RW = 2 * CW + 1, RH = 2 * CH + 1;  // fine residual region
  constexpr int UW = RW + 2, UH = RH + 2;          // fine x region
  __shared__ T su[UH * UW];
  __shared__ T sr[RH * RW];
  const int xcd = blockIdx.x & 7, loc = blockIdx.x >> 3;
  const int t = xcd * a.per + loc;
  if (t >= a.ntx * a.nty) return;
  const int tx = t % a.ntx, ty = t / a.ntx;
  const int cI0 = a.I0 + tx * CW, cJ0 = a.J0 + ty * CH;
  const int fx0 = 2 * cI0 - 1, fy0 = 2 * cJ0 - 1;  // residual region origin
  const int ux0 = fx0 - 1, uy0 = fy0 - 1;
  for (int q = threadIdx.x; q < UW * UH; q += blockDim.x) {
    const int gi = ux0 + q % UW, gj = uy0 + q / UW;
    su[q] = (gi >= 0 && gj >= 0 && gi <= a.N && gj <= a.N) ? a.x[gi + (int64_t)gj * a.s] : T(0);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < RW * RH; q += blockDim.x) {
    const int ri = q % RW, rj = q / RW;
    const int gi = fx0 + ri, gj = fy0 + rj;
    T r = T(0);
    if (gi >= 0 && gj >= 0 && gi <= a.N && gj <= a.N) {
      const int64_t k = gi + (int64_t)gj * a.s;
      const uint8_t f = a.fl[k];
      if (f & kFlagActive) {
        const int sq = (ri + 1) + (rj + 1) * UW;
        T diag;
        const T ax = (f & kFlagStored) ? stored_row<T, UW>(a.A, a.n, k, su, sq, diag)
                                       : q1_row<T, UW>(su, sq, diag);
        r = a.b[k] - ax;
      }
    }
    sr[q] = r;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < CW * CH; q += blockDim.x) {
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
// Coarse levels in one workgroup.  Per level the host packs a descriptor:
//   [0] N  [1] W  [2] H  [3] ox  [4] oy  (LDS box of W x H nodes with origin
//   (ox, oy) = bounding box grown by one ring)  [5] coef offset  [6] slot offset
//   [7..11] cut-list offsets (5)  [12] lds offset of x  [13] of b  [14] of r
//   [15] of flags  [16] of slot  [17] of coef  [18] of cut lists  [19] nstored
// All LDS offsets are in bytes from the dynamic LDS base; the coarsest level
// also holds the inverse of its active block after its coefficient block.
// ---------------------------------------------------------------------------
constexpr int kDesc = 24;

template <class T>
struct CoarseArgs {
  const int* desc;     // kDesc ints per coarse level
  const T* coef;       // compact stored stencils (9 per stored node)
  const int16_t* slot; // per LDS-box node: stored slot, -1 regular, -2 inactive
  const int16_t* cutl; // cut lists in LDS-box indices
  const double* inv;   // coarsest inverse (cn x cn)
  const int16_t* cidx; // coarsest active nodes in LDS-box indices
  int cn;
  int nlev;            // coarse levels handled here (the last one is solved exactly)
  const T* b_top;      // right-hand side of the first coarse level (global)
  T* x_top;            // its solution (global)
  int s_top;           // grid stride of the first coarse level
  int nu1, nu2, eta, reverse, gstar;
};

template <class T>
__device__ inline T lds_row(const int* d, const unsigned char* base, int q, T& diag) {
  const int W = d[1];
  const T* x = reinterpret_cast<const T*>(base + d[12]);
  const int16_t sl = reinterpret_cast<const int16_t*>(base + d[16])[q];
  if (sl >= 0) {
    const T* cf = reinterpret_cast<const T*>(base + d[17]) + 9 * sl;
    diag = cf[4];
    return cf[0] * x[q - W - 1] + cf[1] * x[q - W] + cf[2] * x[q - W + 1] + cf[3] * x[q - 1] +
           cf[4] * x[q] + cf[5] * x[q + 1] + cf[6] * x[q + W - 1] + cf[7] * x[q + W] +
           cf[8] * x[q + W + 1];
  }
  diag = T(8) / T(3);
  const T nb = (x[q - W - 1] + x[q - W] + x[q - W + 1]) + (x[q - 1] + x[q + 1]) +
               (x[q + W - 1] + x[q + W] + x[q + W + 1]);
  return diag * x[q] - nb / T(3);
}

template <class T>
__device__ void wg_smooth(const int* d, unsigned char* base, int eta, bool reverse) {
  const int W = d[1], H = d[2];
  T* x = reinterpret_cast<T*>(base + d[12]);
  const T* b = reinterpret_cast<const T*>(base + d[13]);
  const int16_t* sl = reinterpret_cast<const int16_t*>(base + d[16]);
  const int16_t* cl = reinterpret_cast<const int16_t*>(base + d[18]);
  const int ox = d[3], oy = d[4];
  auto full = [&](int c) {
    const int cx = c & 1, cy = c >> 1;
    const int fx = 1 + ((cx - (ox + 1)) & 1), fy = 1 + ((cy - (oy + 1)) & 1);
    const int nx = (W - 1 - fx + 1) / 2, ny = (H - 1 - fy + 1) / 2;
    for (int q = threadIdx.x; q < nx * ny; q += blockDim.x) {
      const int li = fx + 2 * (q % nx), lj = fy + 2 * (q / nx);
      const int qq = li + lj * W;
      if (sl[qq] == -2) continue;
      T diag;
      const T ax = lds_row<T>(d, base, qq, diag);
      x[qq] += (b[qq] - ax) / diag;
    }
    __syncthreads();
  };
  auto cut = [&](int c) {
    const int lo = d[7 + c] - d[7], hi = d[8 + c] - d[7];
    for (int t = lo + threadIdx.x; t < hi; t += blockDim.x) {
      const int qq = cl[t];
      T diag;
      const T ax = lds_row<T>(d, base, qq, diag);
      x[qq] += (b[qq] - ax) / diag;
    }
    __syncthreads();
  };
  if (!reverse) {
    for (int c = 0; c < 4; ++c) full(c);
    for (int e = 0; e < eta; ++e)
      for (int c = 0; c < 4; ++c) cut(c);
  } else {
    for (int e = 0; e < eta; ++e)
      for (int c = 3; c >= 0; --c) cut(c);
    for (int c = 3; c >= 0; --c) full(c);
  }
}

// restriction of the residual of level d (fine) to level dc (coarse), in LDS
template <class T>
__device__ void wg_restrict(const int* d, const int* dc, unsigned char* base) {
  const int W = d[1], H = d[2];
  T* r = reinterpret_cast<T*>(base + d[14]);
  const T* b = reinterpret_cast<const T*>(base + d[13]);
  const int16_t* sl = reinterpret_cast<const int16_t*>(base + d[16]);
  for (int q = threadIdx.x; q < W * H; q += blockDim.x) {
    const int li = q % W, lj = q / W;
    T rv = T(0);
    if (li > 0 && lj > 0 && li < W - 1 && lj < H - 1 && sl[q] != -2) {
      T diag;
      rv = b[q] - lds_row<T>(d, base, q, diag);
    }
    r[q] = rv;
  }
  __syncthreads();
  const int Wc = dc[1], Hc = dc[2];
  T* xc = reinterpret_cast<T*>(base + dc[12]);
  T* bc = reinterpret_cast<T*>(base + dc[13]);
  const int16_t* slc = reinterpret_cast<const int16_t*>(base + dc[16]);
  for (int q = threadIdx.x; q < Wc * Hc; q += blockDim.x) {
    xc[q] = T(0);
    T v = T(0);
    if (slc[q] != -2) {
      const int I = dc[3] + q % Wc, J = dc[4] + q / Wc;
      const int fi = 2 * I - d[3], fj = 2 * J - d[4];  // centre in the fine LDS box
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          const int li = fi + di, lj = fj + dj;
          if (li < 0 || lj < 0 || li >= W || lj >= H) continue;
          const T w = T((di == 0 ? 1.0 : 0.5) * (dj == 0 ? 1.0 : 0.5));
          v += w * r[li + lj * W];
        }
    }
    bc[q] = v;
  }
  __syncthreads();
}

template <class T>
__device__ void wg_prolong(const int* d, const int* dc, unsigned char* base) {
  const int W = d[1], H = d[2];
  T* x = reinterpret_cast<T*>(base + d[12]);
  const int16_t* sl = reinterpret_cast<const int16_t*>(base + d[16]);
  const int Wc = dc[1];
  const T* xc = reinterpret_cast<const T*>(base + dc[12]);
  for (int q = threadIdx.x; q < W * H; q += blockDim.x) {
    if (sl[q] == -2) continue;
    const int i = d[3] + q % W, j = d[4] + q / W;
    const int I = (i >> 1) - dc[3], J = (j >> 1) - dc[4];
    const int kc = I + J * Wc;
    T val;
    if (!(i & 1) && !(j & 1)) val = xc[kc];
    else if ((i & 1) && !(j & 1)) val = T(0.5) * (xc[kc] + xc[kc + 1]);
    else if (!(i & 1) && (j & 1)) val = T(0.5) * (xc[kc] + xc[kc + Wc]);
    else val = T(0.25) * ((xc[kc] + xc[kc + 1]) + (xc[kc + Wc] + xc[kc + Wc + 1]));
    x[q] += val;
  }
  __syncthreads();
}

template <class T>
__device__ void wg_cycle(const CoarseArgs<T>& a, unsigned char* base, int l) {
  const int* d = a.desc + kDesc * l;
  if (l == a.nlev - 1) {  // exact solve with the stored inverse (float64)
    T* x = reinterpret_cast<T*>(base + d[12]);
    const T* b = reinterpret_cast<const T*>(base + d[13]);
    const double* inv = reinterpret_cast<const double*>(base + d[20]);
    for (int r = threadIdx.x; r < a.cn; r += blockDim.x) {
      double acc = 0.0;
      for (int cc = 0; cc < a.cn; ++cc) acc += inv[r * a.cn + cc] * (double)b[a.cidx[cc]];
      x[a.cidx[r]] = (T)acc;
    }
    __syncthreads();
    return;
  }
  const int* dc = a.desc + kDesc * (l + 1);
  const int pre = a.reverse ? a.nu2 : a.nu1, post = a.reverse ? a.nu1 : a.nu2;
  for (int s = 0; s < pre; ++s) wg_smooth<T>(d, base, a.eta, a.reverse);
  wg_restrict<T>(d, dc, base);
  for (int g = 0; g < a.gstar; ++g) wg_cycle<T>(a, base, l + 1);
  wg_prolong<T>(d, dc, base);
  for (int s = 0; s < post; ++s) wg_smooth<T>(d, base, a.eta, a.reverse);
}

template <class T>
__global__ __launch_bounds__(1024) void k_coarse(CoarseArgs<T> a) {
  extern __shared__ __align__(16) unsigned char base[];
  // stage every coarse level: x = 0, b = 0 (b of the first level from global),
  // flags/slots, stored stencils, cut lists; the inverse of the coarsest block
  for (int l = 0; l < a.nlev; ++l) {
    const int* d = a.desc + kDesc * l;
    const int W = d[1], H = d[2], nb = W * H;
    T* x = reinterpret_cast<T*>(base + d[12]);
    T* b = reinterpret_cast<T*>(base + d[13]);
    int16_t* sl = reinterpret_cast<int16_t*>(base + d[16]);
    T* cf = reinterpret_cast<T*>(base + d[17]);
    int16_t* cl = reinterpret_cast<int16_t*>(base + d[18]);
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
      x[q] = T(0);
      sl[q] = a.slot[d[6] + q];
      T bv = T(0);
      if (l == 0 && sl[q] != -2) {
        const int gi = d[3] + q % W, gj = d[4] + q / W;
        bv = a.b_top[gi + (int64_t)gj * a.s_top];
      }
      b[q] = bv;
    }
    for (int q = threadIdx.x; q < 9 * d[19]; q += blockDim.x) cf[q] = a.coef[9 * (int64_t)d[5] + q];
    const int ncl = d[11] - d[7];
    for (int q = threadIdx.x; q < ncl; q += blockDim.x) cl[q] = a.cutl[d[7] + q];
    if (l == a.nlev - 1) {
      double* inv = reinterpret_cast<double*>(base + d[20]);
      for (int q = threadIdx.x; q < a.cn * a.cn; q += blockDim.x) inv[q] = a.inv[q];
    }
  }
  __syncthreads();
  // gamma* cycles on the first coarse level, each continuing from the last
  for (int g = 0; g < a.gstar; ++g) wg_cycle<T>(a, base, 0);
  const int* d = a.desc;
  const int W = d[1], H = d[2];
  const T* x = reinterpret_cast<const T*>(base + d[12]);
  const int16_t* sl = reinterpret_cast<const int16_t*>(base + d[16]);
  for (int q = threadIdx.x; q < W * H; q += blockDim.x) {
    if (sl[q] == -2) continue;
    const int gi = d[3] + q % W, gj = d[4] + q / W;
    a.x_top[gi + (int64_t)gj * a.s_top] = x[q];
  }
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

template <class T, int TW, int TH>
void launch_sweep(mgfem_ctx* c, int l, bool reverse) {
  Level& L = c->lv[l];
  SweepArgs<T> a;
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
  const int tiles = a.ntx * a.nty;
  a.per = (tiles + 7) / 8;
  a.reverse = reverse ? 1 : 0;
  hipLaunchKernelGGL((k_sweep<T, TW, TH>), dim3(8 * a.per), dim3(256), 0, c->s, a);
  L.cur = 1 - L.cur;
}

template <class T>
void sweep(mgfem_ctx* c, int l, bool reverse) {
  Level& L = c->lv[l];
  if (L.empty()) return;
  if (L.N >= 1024) launch_sweep<T, 64, 32>(c, l, reverse);
  else launch_sweep<T, 32, 16>(c, l, reverse);
}

template <class T>
void cut_sweeps(mgfem_ctx* c, int l, bool reverse) {
  Level& L = c->lv[l];
  const int eta = c->p.eta;
  if (eta == 0 || L.cut_off[4] == 0) return;
  if (L.cp.ok) {
    CutArgs<T> a;
    a.g_info = L.cp.g_info;
    a.cl_node = L.cp.cl_node;
    a.cl_q = L.cp.cl_q;
    a.cl_own = L.cp.cl_own;
    a.cl_nbr = L.cp.cl_nbr;
    a.ext_src = L.cp.ext_src;
    a.x = Xp<T>(L, L.cur);
    a.b = Bp<T>(L);
    a.A = Ap<T>(L);
    a.snap = Sp<T>(L);
    a.n = L.n;
    a.eta = eta;
    a.reverse = reverse ? 1 : 0;
    const size_t lds = (size_t)L.cp.max_cl * (11 * sizeof(T) + 16) + (size_t)L.cp.max_ext * sizeof(T) + 16;
    hipLaunchKernelGGL(k_cut<T>, dim3(L.cp.ngroups), dim3(256), lds, c->s, a);
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
void launch_resrestrict(mgfem_ctx* c, int l) {
  Level& L = c->lv[l];
  Level& C = c->lv[l + 1];
  if (C.empty()) return;
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
  a.per = (a.ntx * a.nty + 7) / 8;
  hipLaunchKernelGGL((k_resrestrict<T, CW, CH>), dim3(8 * a.per), dim3(256), 0, c->s, a);
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

template <class T>
void coarse_wg(mgfem_ctx* c, bool reverse) {
  CoarsePlan& P = c->cplan;
  Level& Lc = c->lv[P.lc];
  CoarseArgs<T> a;
  const bool f32 = !std::is_same<T, double>::value;
  a.desc = P.desc + (f32 ? kDesc * P.ndesc : 0);
  a.coef = std::is_same<T, double>::value ? reinterpret_cast<const T*>(P.coef)
                                          : reinterpret_cast<const T*>(P.coef32);
  a.slot = P.slot;
  a.cutl = P.cutl;
  a.inv = P.inv;
  a.cidx = reinterpret_cast<const int16_t*>(P.desc + 2 * kDesc * P.ndesc);
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
  const int lds = std::is_same<T, double>::value ? P.lds64 : P.lds32;
  hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(1024), lds, c->s, a);
  Lc.cur = 0;
}

template <class T>
void cycle_level(mgfem_ctx* c, int l, bool reverse) {
  const int nl = (int)c->lv.size();
  if (c->cplan.lc >= 0 && l == c->cplan.lc) {
    coarse_wg<T>(c, reverse);
    return;
  }
  if (l == nl - 1) return;  // unreachable: the coarse plan always covers the coarsest level
  const int pre = reverse ? c->p.nu2 : c->p.nu1;
  const int post = reverse ? c->p.nu1 : c->p.nu2;
  for (int s = 0; s < pre; ++s) smooth<T>(c, l, reverse);
  if (c->lv[l].N >= 1024) launch_resrestrict<T, 32, 16>(c, l);
  else launch_resrestrict<T, 16, 8>(c, l);
  const int gstar = c->p.cycle == MGFEM_CYCLE_W ? 2 : 1;
  if (l + 1 == c->cplan.lc) coarse_wg<T>(c, reverse);  // runs its gamma* cycles itself
  else
    for (int g = 0; g < gstar; ++g) cycle_level<T>(c, l + 1, reverse);
  prolong<T>(c, l);
  for (int s = 0; s < post; ++s) smooth<T>(c, l, reverse);
}

}  // namespace

void run_cycle(mgfem_ctx* c, const CycleOpts& o) {
  if (o.fp32) cycle_level<float>(c, 0, o.reverse);
  else cycle_level<double>(c, 0, o.reverse);
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
