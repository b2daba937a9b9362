// Setup on the device, part 2: the Galerkin hierarchy and its bookkeeping.
//
// Coarse operators A_{l+1} = R A_l P with P the bilinear prolongation of the
// exact shape-function relation (section 5.1) and R = P^T (eq. galerkin,
// read with the operators in the order that makes the product square).  Each
// coarse row is gathered from the nine fine rows in the support of its coarse
// shape function, so the product needs no atomics and is deterministic.
// A coarse node is active when its diagonal is non-zero.  A coarse row is the
// constant interior Q1 stencil when all nine fine rows it is built from are
// (shape functions are nested); such rows are marked as not stored.
// Cut cells of a coarse grid are those containing a cut fine cell; their
// vertices form the extra-smoothing set of that level (every level but the
// coarsest).  The coarsest active block is factored by Cholesky.
#include <algorithm>
#include <cmath>

#include "mgfem_internal.h"

namespace mgfem {
namespace {

__device__ inline double pw(int d) { return d == 0 ? 1.0 : 0.5; }  // 1D prolongation weight

__global__ void k_rap(const double* __restrict__ Af, const uint8_t* __restrict__ flf, int Nf,
                      double* __restrict__ Ac, uint8_t* __restrict__ flc, int Nc) {
  const int sf = Nf + 1, sc = Nc + 1;
  const int64_t nf = (int64_t)sf * sf, nc = (int64_t)sc * sc;
  int64_t kc = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (kc >= nc) return;
  const int I = (int)(kc % sc), J = (int)(kc / sc);
  double acc[9];
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  bool regular = true;
  for (int b = -1; b <= 1; ++b)
    for (int a = -1; a <= 1; ++a) {
      const int fi = 2 * I + a, fj = 2 * J + b;
      if (fi < 0 || fj < 0 || fi > Nf || fj > Nf) {
        regular = false;
        continue;
      }
      const int64_t fk = fi + (int64_t)fj * sf;
      const uint8_t fl = flf[fk];
      if ((fl & kFlagStored) || !(fl & kFlagActive)) regular = false;
      if (!(fl & kFlagActive)) continue;
      const double wi = pw(a) * pw(b);
      for (int ey = -1; ey <= 1; ++ey)
        for (int ex = -1; ex <= 1; ++ex) {
          const double aij = Af[((ex + 1) + 3 * (ey + 1)) * nf + fk];
          if (aij == 0.0) continue;
          const int gi = fi + ex, gj = fj + ey;  // column node j
          for (int dy = -1; dy <= 1; ++dy) {
            const int py = gj - 2 * (J + dy);
            if (py < -1 || py > 1 || J + dy < 0 || J + dy > Nc) continue;
            for (int dx = -1; dx <= 1; ++dx) {
              const int px = gi - 2 * (I + dx);
              if (px < -1 || px > 1 || I + dx < 0 || I + dx > Nc) continue;
              acc[(dx + 1) + 3 * (dy + 1)] += wi * aij * (pw(px) * pw(py));
            }
          }
        }
    }
  for (int q = 0; q < 9; ++q) Ac[q * nc + kc] = acc[q];
  uint8_t f = 0;
  if (acc[4] != 0.0) {
    f |= kFlagActive;
    if (!regular) f |= kFlagStored;
  }
  flc[kc] = f;
}

__global__ void k_coarsen_cells(const uint8_t* __restrict__ cf, int Nf, uint8_t* __restrict__ cc,
                                int Nc) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= (int64_t)Nc * Nc) return;
  int I = (int)(c % Nc), J = (int)(c / Nc);
  int64_t f0 = 2 * I + (int64_t)(2 * J) * Nf;
  cc[c] = (cf[f0] | cf[f0 + 1] | cf[f0 + Nf] | cf[f0 + Nf + 1]) ? 1 : 0;
}

// mark vertices of cut cells (active ones) and accumulate the active bounding box
__global__ void k_mark_cut_bbox(const uint8_t* __restrict__ cellcut, int N, uint8_t* __restrict__ fl,
                                int mark, int* __restrict__ bbox) {
  const int s = N + 1;
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= (int64_t)s * s) return;
  int i = (int)(k % s), j = (int)(k / s);
  uint8_t f = fl[k];
  if (!(f & kFlagActive)) return;
  if (mark) {
    bool cut = false;
    for (int cy = j - 1; cy <= j; ++cy)
      for (int cx = i - 1; cx <= i; ++cx)
        if (cx >= 0 && cy >= 0 && cx < N && cy < N && cellcut[cx + (int64_t)cy * N]) cut = true;
    if (cut) fl[k] = f | kFlagCut;
  }
  atomicMin(&bbox[0], i);
  atomicMax(&bbox[1], i);
  atomicMin(&bbox[2], j);
  atomicMax(&bbox[3], j);
}

// ordered compaction of the cut vertices, one list per colour, by rows
__global__ void k_row_count(const uint8_t* __restrict__ fl, int N, int j0, int j1, int i0, int i1,
                            int* __restrict__ cnt /* 4 x (N+1) */) {
  int j = j0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (j > j1) return;
  const int s = N + 1;
  int c4[4] = {0, 0, 0, 0};
  for (int i = i0; i <= i1; ++i)
    if (fl[i + (int64_t)j * s] & kFlagCut) ++c4[(i & 1) + 2 * (j & 1)];
  for (int c = 0; c < 4; ++c) cnt[c * s + j] = c4[c];
}

__global__ void k_row_scan(int* __restrict__ cnt, int N, int* __restrict__ tot /* 5 */) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int s = N + 1;
  int base = 0;
  for (int c = 0; c < 4; ++c) {
    tot[c] = base;
    for (int j = 0; j < s; ++j) {
      int v = cnt[c * s + j];
      cnt[c * s + j] = base;
      base += v;
    }
  }
  tot[4] = base;
}

__global__ void k_row_scatter(const uint8_t* __restrict__ fl, int N, int j0, int j1, int i0, int i1,
                              const int* __restrict__ off, int* __restrict__ list) {
  int j = j0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (j > j1) return;
  const int s = N + 1;
  int pos[4];
  for (int c = 0; c < 4; ++c) pos[c] = off[c * s + j];
  for (int i = i0; i <= i1; ++i) {
    int64_t k = i + (int64_t)j * s;
    if (fl[k] & kFlagCut) list[pos[(i & 1) + 2 * (j & 1)]++] = (int)k;
  }
}

// gather and factor the coarsest active block (one thread: at most a few hundred unknowns)
__global__ void k_coarse_factor(const double* __restrict__ A, const uint8_t* __restrict__ fl, int N,
                                double* __restrict__ Lm, int* __restrict__ idx, double* __restrict__ inv,
                                Stats* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int s = N + 1;
  const int64_t n = (int64_t)s * s;
  int cn = 0;
  for (int64_t k = 0; k < n; ++k)
    if (fl[k] & kFlagActive) idx[cn++] = (int)k;
  for (int r = 0; r < cn * cn; ++r) Lm[r] = 0.0;
  for (int r = 0; r < cn; ++r) {
    const int k = idx[r];
    for (int p = 0; p < 9; ++p) {
      const double v = A[p * n + k];
      if (v == 0.0) continue;
      const int kk = k + (p % 3 - 1) + (p / 3 - 1) * s;
      for (int q = 0; q < cn; ++q)
        if (idx[q] == kk) Lm[r * cn + q] = v;
    }
  }
  int status = 0;
  for (int j = 0; j < cn; ++j) {
    double d = Lm[j * cn + j];
    for (int t = 0; t < j; ++t) d -= Lm[j * cn + t] * Lm[j * cn + t];
    if (!(d > 0.0)) {
      status = 1;
      break;
    }
    d = sqrt(d);
    Lm[j * cn + j] = d;
    for (int i = j + 1; i < cn; ++i) {
      double v = Lm[i * cn + j];
      for (int t = 0; t < j; ++t) v -= Lm[i * cn + t] * Lm[j * cn + t];
      Lm[i * cn + j] = v / d;
    }
  }
  st->coarse_status = status;
  st->coarse_n = cn;
  if (status) return;
  // explicit inverse A^{-1} = L^{-T} L^{-1}, one column at a time
  for (int col = 0; col < cn; ++col) {
    double* x = inv + (int64_t)col * cn;  // column stored as a row (A^{-1} is symmetric)
    for (int i = 0; i < cn; ++i) {
      double v = (i == col) ? 1.0 : 0.0;
      for (int t = 0; t < i; ++t) v -= Lm[i * cn + t] * x[t];
      x[i] = v / Lm[i * cn + i];
    }
    for (int i = cn - 1; i >= 0; --i) {
      double v = x[i];
      for (int t = i + 1; t < cn; ++t) v -= Lm[t * cn + i] * x[t];
      x[i] = v / Lm[i * cn + i];
    }
  }
}

__global__ void k_count_flags(const uint8_t* __restrict__ fl, int64_t n, unsigned long long* __restrict__ out) {
  __shared__ unsigned int ca, cs;
  if (threadIdx.x == 0) ca = cs = 0;
  __syncthreads();
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) {
    const uint8_t f = fl[k];
    if (f & kFlagActive) atomicAdd(&ca, 1u);
    if ((f & kFlagActive) && (f & kFlagStored)) atomicAdd(&cs, 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (ca) atomicAdd(&out[0], (unsigned long long)ca);
    if (cs) atomicAdd(&out[1], (unsigned long long)cs);
  }
}

__global__ void k_to_float(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) dst[k] = (float)src[k];
}

inline unsigned nblk(int64_t n, int tb) { return (unsigned)((n + tb - 1) / tb); }

}  // namespace

int setup_hierarchy(mgfem_ctx* c, const double* psi_in, const double* chi_in) {
  const int tb = 256;
  const int nl = (int)c->lv.size();
  const bool mixed = c->p.precision == MGFEM_PREC_MIXED;
  // coarse operators
  for (int l = 0; l + 1 < nl; ++l) {
    Level& F = c->lv[l];
    Level& C = c->lv[l + 1];
    if (c->p.coarse_op == MGFEM_COARSE_REDISCRETISED) {
      const int rc = assemble_level(c, l + 1, psi_in, chi_in);
      if (rc != MGFEM_OK) return rc;
      continue;
    }
    MGFEM_HIP_TRY(ctx_alloc_t(c, &C.A, 9 * C.n));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &C.flags, C.n));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &C.cellcut, (int64_t)C.N * C.N));
    hipLaunchKernelGGL(k_rap, dim3(nblk(C.n, tb)), dim3(tb), 0, c->s, F.A, F.flags, F.N, C.A,
                       C.flags, C.N);
    hipLaunchKernelGGL(k_coarsen_cells, dim3(nblk((int64_t)C.N * C.N, tb)), dim3(tb), 0, c->s,
                       F.cellcut, F.N, C.cellcut, C.N);
  }
  MGFEM_HIP_TRY(hipGetLastError());
  // cut marks, bounding boxes, work vectors
  int* bb = nullptr;
  MGFEM_HIP_TRY(ctx_alloc_t(c, &bb, 4 * nl));
  std::vector<int> bbh(4 * nl);
  for (int l = 0; l < nl; ++l) {
    bbh[4 * l + 0] = 1 << 30;
    bbh[4 * l + 1] = -1;
    bbh[4 * l + 2] = 1 << 30;
    bbh[4 * l + 3] = -1;
  }
  MGFEM_HIP_TRY(hipMemcpyAsync(bb, bbh.data(), 4 * nl * sizeof(int), hipMemcpyHostToDevice, c->s));
  for (int l = 0; l < nl; ++l) {
    Level& L = c->lv[l];
    hipLaunchKernelGGL(k_mark_cut_bbox, dim3(nblk(L.n, tb)), dim3(tb), 0, c->s, L.cellcut, L.N,
                       L.flags, (l + 1 < nl) ? 1 : 0, bb + 4 * l);
  }
  MGFEM_HIP_TRY(hipGetLastError());
  MGFEM_HIP_TRY(hipMemcpyAsync(bbh.data(), bb, 4 * nl * sizeof(int), hipMemcpyDeviceToHost, c->s));
  MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
  for (int l = 0; l < nl; ++l) {
    Level& L = c->lv[l];
    for (int q = 0; q < 4; ++q) L.bbox[q] = bbh[4 * l + q];
    if (L.bbox[1] < 0) {  // empty level
      L.bbox[0] = 1;
      L.bbox[1] = 0;
      L.bbox[2] = 1;
      L.bbox[3] = 0;
    }
  }
  if (c->lv[0].empty()) {
    c->last_error = "no active node: the level set has no point with psi < 0 after snapping";
    return MGFEM_ERR_EMPTY_DOMAIN;
  }
  // active and stored row counts per level
  {
    unsigned long long* cntd = nullptr;
    MGFEM_HIP_TRY(ctx_alloc_t(c, &cntd, 2 * nl));
    for (int l = 0; l < nl; ++l)
      hipLaunchKernelGGL(k_count_flags, dim3(nblk(c->lv[l].n, tb)), dim3(tb), 0, c->s, c->lv[l].flags, c->lv[l].n,
                         cntd + 2 * l);
    std::vector<unsigned long long> h(2 * nl);
    MGFEM_HIP_TRY(hipMemcpyAsync(h.data(), cntd, 2 * nl * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->s));
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
    for (int l = 0; l < nl; ++l) {
      c->lv[l].n_active = (int64_t)h[2 * l];
      c->lv[l].n_stored = (int64_t)h[2 * l + 1];
    }
  }
  // cut lists
  int* cnt = nullptr;
  int* tot = nullptr;
  MGFEM_HIP_TRY(ctx_alloc_t(c, &cnt, 4 * (c->lv[0].stride)));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &tot, 5));
  for (int l = 0; l + 1 < nl; ++l) {
    Level& L = c->lv[l];
    MGFEM_HIP_TRY(hipMemsetAsync(cnt, 0, 4 * L.stride * sizeof(int), c->s));
    const int j0 = L.bbox[2], j1 = L.bbox[3], i0 = L.bbox[0], i1 = L.bbox[1];
    const unsigned nb = nblk(j1 - j0 + 1, 64);
    hipLaunchKernelGGL(k_row_count, dim3(nb), dim3(64), 0, c->s, L.flags, L.N, j0, j1, i0, i1, cnt);
    hipLaunchKernelGGL(k_row_scan, dim3(1), dim3(1), 0, c->s, cnt, L.N, tot);
    int toth[5];
    MGFEM_HIP_TRY(hipMemcpyAsync(toth, tot, 5 * sizeof(int), hipMemcpyDeviceToHost, c->s));
    MGFEM_HIP_TRY(hipStreamSynchronize(c->s));
    for (int q = 0; q < 5; ++q) L.cut_off[q] = toth[q];
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.cut_list, std::max(1, toth[4])));
    hipLaunchKernelGGL(k_row_scatter, dim3(nb), dim3(64), 0, c->s, L.flags, L.N, j0, j1, i0, i1,
                       cnt, L.cut_list);
    MGFEM_HIP_TRY(hipGetLastError());
  }
  // work vectors (zero-initialised: inactive entries are read but never written)
  for (int l = 0; l < nl; ++l) {
    Level& L = c->lv[l];
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.X[0], L.n));
    if (l > 0) MGFEM_HIP_TRY(ctx_alloc_t(c, &L.b, L.n));
    MGFEM_HIP_TRY(ctx_alloc_t(c, &L.X[1], L.n));
    if (l == 0) c->x0 = L.X[0];
    if (mixed) {
      MGFEM_HIP_TRY(ctx_alloc_t(c, &L.A32, 9 * L.n));
      hipLaunchKernelGGL(k_to_float, dim3(nblk(9 * L.n, tb)), dim3(tb), 0, c->s, L.A, L.A32,
                         9 * L.n);
      MGFEM_HIP_TRY(ctx_alloc_t(c, &L.X32[0], L.n));
      MGFEM_HIP_TRY(ctx_alloc_t(c, &L.X32[1], L.n));
      MGFEM_HIP_TRY(ctx_alloc_t(c, &L.b32, L.n));
    }
  }
  // coarsest factorisation
  Level& Lc = c->lv[nl - 1];
  const int cmax = (int)Lc.n;
  MGFEM_HIP_TRY(ctx_alloc_t(c, &c->coarse_L, (int64_t)cmax * cmax));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &c->coarse_idx, cmax));
  MGFEM_HIP_TRY(ctx_alloc_t(c, &c->cplan.inv, (int64_t)cmax * cmax));
  hipLaunchKernelGGL(k_coarse_factor, dim3(1), dim3(64), 0, c->s, Lc.A, Lc.flags, Lc.N, c->coarse_L,
                     c->coarse_idx, c->cplan.inv, c->stats);
  MGFEM_HIP_TRY(hipGetLastError());
  return MGFEM_OK;
}

}  // namespace mgfem
