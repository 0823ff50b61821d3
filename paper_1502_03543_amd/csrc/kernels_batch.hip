// Batched Primal-Dual Affine Scaling: many independent LPs of their own
// shapes (m_i, n_i), each advanced by the Section 3 iteration (Section 5
// normal equations, Cholesky of Section 5.1).
//
// One launch per iteration for the whole batch.  Workgroups take LPs from an
// atomic queue (largest m^2 n first, so the long ones start early) until the
// queue is empty; a workgroup owns its LP for every phase of the iteration,
// so no grid-wide synchronisation exists and every workgroup ends when the
// queue runs dry.
//
// Phases (all inside one workgroup of 256 threads, barriers between them):
//   d = x/s, w = d o r_d; rhs = b + A w            (wavefront per row)
//   M = A D A^T, lower 64 x 64 tiles               (FP64 MFMA 4x4x4, LDS-staged)
//   Cholesky, 64-wide panels: diagonal block and panel solve in LDS,
//     trailing update with the same MFMA tile routine (subtract mode)
//   L z = rhs, L^T dy = z                          (64-row blocks, readlane solves)
//   g = A^T dy, g_y = A^T y; ds, dx; psi (first maximiser); step; next r_d; gap
// Per-LP status words mirror the single-LP statuses.
#include <climits>
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

constexpr int BT = 64;   // tile / panel width
constexpr int BKC = 16;  // K per LDS stage of the tile routine

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double rl(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__device__ inline void amerge(double& v, long long& i, double v2, long long i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// LDS layout of a 64 x BKC stage (blocks of 4 k by 16 rows, lane-linear reads).
__device__ inline int bidx(int row, int k) {
  return (((k >> 2) * (BT / 16) + (row >> 4)) << 6) + ((k & 3) << 4) + (row & 15);
}

// One 64 x 64 tile of C (row-major, ldc) at (row0, col0):
//   C = X_r diag(w) X_c^T  (sub = false)   or   C -= X_r X_c^T  (sub = true),
// X rows of length K (stride ldx), rows limited to mm.  Lower part of
// diagonal tiles only.  All 256 threads participate; 2 x 2 wavefronts of
// 32 x 32 (v_mfma_f64_4x4x4_4b: A lane x+4blk+16y = rowop[x][y], B = colop
// [4blk + x][y], D = C[y][4blk + x]).  lds: 2 * 2 * 64 * BKC doubles.
__device__ void tile_syrk(int mm, int K, const double* __restrict__ X, long ldx,
                          const double* __restrict__ w, double* C, long ldc, int row0, int col0,
                          bool sub, double* lds) {
  constexpr int R = 8, Q = 2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int x = lane & 3, blk = (lane >> 2) & 3, y = lane >> 4;
  const int wr0 = (wv >> 1) * 32, wc0 = (wv & 1) * 32;
  const bool diag = row0 == col0;
  const bool active = !(diag && wr0 + 32 <= wc0);
  double acc[R][Q];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[r][q] = 0.0;
  // each thread stages 2 pairs per operand per stage (64 rows x 16 k)
  const int nst = (K + BKC - 1) / BKC;
  double2 pa[2], pb[2], pw[2];
  auto gload = [&](int st) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int p = tid + 256 * it;
      const int row = p >> 3, k = st * BKC + 2 * (p & 7);
      const long ra = min(row0 + row, mm - 1), rb = min(col0 + row, mm - 1);
      const int k0 = min(k, K - 1), k1 = min(k + 1, K - 1);
      pa[it].x = X[ra * ldx + k0];
      pa[it].y = X[ra * ldx + k1];
      pb[it].x = X[rb * ldx + k0];
      pb[it].y = X[rb * ldx + k1];
      if (w) {
        pw[it].x = w[k0];
        pw[it].y = w[k1];
      }
    }
  };
  auto sstore = [&](int buf, int st) {
    double* la = lds + buf * (2 * BT * BKC);
    double* lb = la + BT * BKC;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int p = tid + 256 * it;
      const int row = p >> 3, kk = 2 * (p & 7), k = st * BKC + kk;
      const bool va = row0 + row < mm, vb = col0 + row < mm;
      double a0 = pa[it].x, a1 = pa[it].y;
      if (w) {
        a0 *= pw[it].x;
        a1 *= pw[it].y;
      }
      la[bidx(row, kk)] = (va && k < K) ? a0 : 0.0;
      la[bidx(row, kk + 1)] = (va && k + 1 < K) ? a1 : 0.0;
      lb[bidx(row, kk)] = (vb && k < K) ? pb[it].x : 0.0;
      lb[bidx(row, kk + 1)] = (vb && k + 1 < K) ? pb[it].y : 0.0;
    }
  };
  if (nst > 0) {
    gload(0);
    sstore(0, 0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) gload(st + 1);
    if (active) {
      const double* la = lds + cur * (2 * BT * BKC);
      const double* lb = la + BT * BKC;
#pragma unroll
      for (int ks = 0; ks < BKC / 4; ++ks) {
        double bq[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) bq[q] = lb[bidx(wc0 + 16 * q + 4 * blk + x, 4 * ks + y)];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double av = la[bidx(wr0 + 4 * r + x, 4 * ks + y)];
#pragma unroll
          for (int q = 0; q < Q; ++q)
            acc[r][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bq[q], acc[r][q], 0, 0, 0);
        }
      }
    }
    if (st + 1 < nst) sstore(cur ^ 1, st + 1);
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int gr = row0 + wr0 + 4 * r + y, gc = col0 + wc0 + 16 * q + 4 * blk + x;
        if (gr < mm && gc < mm && (!diag || gc <= gr)) {
          double* cp = C + (long)gr * ldc + gc;
          *cp = sub ? (*cp - acc[r][q]) : acc[r][q];
        }
      }
  }
  __syncthreads();
}

// Lower triangle of X diag(w) X^T (sub: C -= X X^T) over all 64-tiles.
__device__ void wg_syrk(int mm, int K, const double* X, long ldx, const double* w, double* C,
                        long ldc, bool sub, double* lds) {
  const int nt = (mm + BT - 1) / BT;
  for (int ti = 0; ti < nt; ++ti)
    for (int tj = 0; tj <= ti; ++tj)
      tile_syrk(mm, K, X, ldx, w, C, ldc, ti * BT, tj * BT, sub, lds);
}

#define PDAS_BSEL16(v, idx)                                                                 \
  ((idx) == 0 ? (v)[0] : (idx) == 1 ? (v)[1] : (idx) == 2 ? (v)[2] : (idx) == 3 ? (v)[3]   \
   : (idx) == 4 ? (v)[4] : (idx) == 5 ? (v)[5] : (idx) == 6 ? (v)[6] : (idx) == 7 ? (v)[7] \
   : (idx) == 8 ? (v)[8] : (idx) == 9 ? (v)[9] : (idx) == 10 ? (v)[10]                      \
   : (idx) == 11 ? (v)[11] : (idx) == 12 ? (v)[12] : (idx) == 13 ? (v)[13]                  \
   : (idx) == 14 ? (v)[14] : (v)[15])

// In-place Cholesky of the lower triangle of M (m x m, row-major, ld) by one
// workgroup.  Returns the first failing column or -1; *minp the smallest
// accepted pivot.  lds: at least 2*64 + 64*65 + 64 doubles (shares the tile
// routine's buffer).
__device__ int wg_potrf(int m, double* M, long ld, double* lds, double* minp_out) {
  double* col = lds;                  // [2][64]
  double* l = lds + 2 * BT;           // [64][65]
  double* dinv = l + BT * (BT + 1);   // [64]
  __shared__ int s_fail;
  __shared__ double s_minp;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_fail = -1;
    s_minp = INFINITY;
  }
  __syncthreads();
  for (int p = 0; p < m; p += BT) {
    const int nbe = min(BT, m - p);
    const int i = tid & 63, g = tid >> 6;
    double a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int k = g + 4 * c;
      double v = (i == k) ? 1.0 : 0.0;
      if (i < nbe && k <= i) v = M[(long)(p + i) * ld + p + k];
      a[c] = v;
    }
    if (g == 0) col[i] = a[0];
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < BT; ++j) {
      const double* cj = col + (j & 1) * BT;
      const double piv = cj[j];
      const double ci = cj[i];
      if (tid == 0 && j < nbe) {
        if (s_fail < 0 && !(piv > 0.0 && isfinite(piv))) s_fail = p + j;
        if (piv < s_minp) s_minp = piv;
      }
      const double ljj = sqrt(piv);
      const double rinv = 1.0 / ljj;
      const double li = ci * rinv;
      if (g == 0) {
        if (i > j) l[i * (BT + 1) + j] = li;
        if (i == j) {
          l[j * (BT + 1) + j] = ljj;
          dinv[j] = rinv;
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int k = g + 4 * c;
        const double upd = a[c] - li * (cj[k] * rinv);
        a[c] = (k > j && k <= i) ? upd : a[c];
      }
      if (j + 1 < BT && g == ((j + 1) & 3)) col[((j + 1) & 1) * BT + i] = PDAS_BSEL16(a, (j + 1) >> 2);
      __syncthreads();
    }
    for (int e = tid; e < BT * BT; e += 256) {
      const int r = e / BT, k = e % BT;
      if (r < nbe && k <= r) M[(long)(p + r) * ld + p + k] = l[r * (BT + 1) + k];
    }
    // panel solve for all rows below, 64 rows at a time (4 lanes per row)
    const int qbase = (tid & 63) & ~3;
    for (int r0 = p + BT; r0 < m; r0 += BT) {
      const int nrow = min(BT, m - r0);
      const int r = tid >> 2, q = tid & 3;
      double xv[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) xv[c] = (r < nrow) ? M[(long)(r0 + r) * ld + p + q + 4 * c] : 0.0;
#pragma unroll 1
      for (int cc = 0; cc < BT; ++cc) {
        const int qo = cc & 3, co = cc >> 2;
        const double xf = __shfl(PDAS_BSEL16(xv, co) * dinv[cc], qbase + qo, 64);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int k = q + 4 * c;
          const double upd = xv[c] - xf * l[k * (BT + 1) + cc];
          xv[c] = (k == cc) ? xf : ((k > cc) ? upd : xv[c]);
        }
      }
      if (r < nrow) {
#pragma unroll
        for (int c = 0; c < 16; ++c) M[(long)(r0 + r) * ld + p + q + 4 * c] = xv[c];
      }
    }
    __syncthreads();
    if (p + BT < m) {
      // trailing update M22 -= L21 L21^T (the tile routine reuses lds)
      wg_syrk(m - p - BT, BT, M + (long)(p + BT) * ld + p, ld, nullptr,
              M + (long)(p + BT) * ld + p + BT, ld, true, lds);
    }
    __syncthreads();
  }
  *minp_out = s_minp;
  const int f = s_fail;
  __syncthreads();
  return f;
}

// z = L^-1 r (forward) into out; L row-major lower with ld.  One workgroup:
// per 64-row block, all threads form the off-diagonal product and stage the
// diagonal block in LDS, then wave 0 solves it with readlane broadcasts.
__device__ void wg_trsv_fwd(int m, const double* L, long ld, const double* r, double* out,
                            double* lds) {
  double* sacc = lds;           // [64]
  double* Ld = lds + BT;        // [64][65]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i0 = 0; i0 < m; i0 += BT) {
    const int rows = min(BT, m - i0);
    for (int e = tid; e < BT * BT; e += 256) {
      const int ii = e / BT, k = e % BT;
      double v = (ii == k) ? 1.0 : 0.0;
      if (ii < rows && k <= ii) v = L[(long)(i0 + ii) * ld + i0 + k];
      Ld[ii * (BT + 1) + k] = v;
    }
    // wave wv: rows wv, wv+4, ...; lanes over columns 0..i0-1
    for (int ii = wv; ii < BT; ii += 4) {
      double acc = 0.0;
      if (ii < rows)
        for (int c = lane; c < i0; c += 64) acc += L[(long)(i0 + ii) * ld + c] * out[c];
      acc = wsum(acc);
      if (lane == 0) sacc[ii] = acc;
    }
    __syncthreads();
    if (wv == 0) {
      const double dl = 1.0 / Ld[lane * (BT + 1) + lane];
      double val = (lane < rows) ? (r[i0 + lane] - sacc[lane]) : 0.0;
      double mine = 0.0;
#pragma unroll 4
      for (int j = 0; j < BT; ++j) {
        const double lij = Ld[lane * (BT + 1) + j];
        const double zj = rl(val, j) * rl(dl, j);
        if (lane == j) mine = zj;
        if (lane > j) val -= lij * zj;
      }
      if (lane < rows) out[i0 + lane] = mine;
    }
    __syncthreads();
  }
}

// y = L^-T z into out.
__device__ void wg_trsv_bwd(int m, const double* L, long ld, const double* z, double* out,
                            double* lds) {
  double* sacc = lds;           // [4][64]
  double* Ld = lds + 4 * BT;    // [64][65]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nblk = (m + BT - 1) / BT;
  for (int rb = nblk - 1; rb >= 0; --rb) {
    const int c0 = rb * BT, cols = min(BT, m - c0);
    for (int e = tid; e < BT * BT; e += 256) {
      const int ii = e / BT, k = e % BT;
      double v = (ii == k) ? 1.0 : 0.0;
      if (ii < cols && k <= ii) v = L[(long)(c0 + ii) * ld + c0 + k];
      Ld[ii * (BT + 1) + k] = v;
    }
    double acc = 0.0;
    if (lane < cols)
      for (int i = c0 + BT + wv; i < m; i += 4) acc += L[(long)i * ld + c0 + lane] * out[i];
    sacc[wv * BT + lane] = acc;
    __syncthreads();
    if (wv == 0) {
      const double dl = 1.0 / Ld[lane * (BT + 1) + lane];
      const double tot = ((sacc[lane] + sacc[BT + lane]) + sacc[2 * BT + lane]) + sacc[3 * BT + lane];
      double val = (lane < cols) ? (z[c0 + lane] - tot) : 0.0;
      double mine = 0.0;
#pragma unroll 4
      for (int j = BT - 1; j >= 0; --j) {
        const double lji = Ld[j * (BT + 1) + lane];
        const double yj = rl(val, j) * rl(dl, j);
        if (lane == j) mine = yj;
        if (lane < j) val -= lji * yj;
      }
      if (lane < cols) out[c0 + lane] = mine;
    }
    __syncthreads();
  }
}

// Block reductions (256 threads); results valid in every thread.
__device__ double bsum(double v, double* sh) {
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;
}

__device__ void bargmax(double& v, long long& i, double* shv, long long* shi) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) amerge(v, i, __shfl_xor(v, o, 64), __shfl_xor(i, o, 64));
  if ((threadIdx.x & 63) == 0) {
    shv[threadIdx.x >> 6] = v;
    shi[threadIdx.x >> 6] = i;
  }
  __syncthreads();
  v = shv[0];
  i = shi[0];
  for (int k = 1; k < 4; ++k) amerge(v, i, shv[k], shi[k]);
  __syncthreads();
}

}  // namespace

// Pointers of one LP inside the batch pools.
struct LPView {
  int m, n;
  long ldm;
  const double *A, *b, *c;
  double *d, *w, *g, *gy, *dx, *ds, *rhs, *z, *dy, *M;
};

__device__ inline LPView lp_view(const BatchArgs& a, const BatchLP& P) {
  LPView v;
  v.m = P.m;
  v.n = P.n;
  v.ldm = P.ldm;
  v.A = a.A + P.a_off;
  v.b = a.b + P.vm;
  v.c = a.c + P.vn;
  v.d = a.d + P.vn;
  v.w = a.w + P.vn;
  v.g = a.g + P.vn;
  v.gy = a.gy + P.vn;
  v.dx = a.dx + P.vn;
  v.ds = a.ds + P.vn;
  v.rhs = a.rhs + P.vm;
  v.z = a.z + P.vm;
  v.dy = a.dy + P.vm;
  v.M = a.M + P.M_off;
  return v;
}

// The direction of one step from (x, y, s, r_d), by the whole workgroup:
// d, w, rhs, M = A D A^T, its Cholesky factor, dy, g = A^T dy, g_y = A^T y,
// ds, dx and the ratio test.  Returns a status (LP_OK, LP_ERR_BREAKDOWN,
// LP_OPTIMAL_ZERO_DIR, LP_ERR_NONPOS_PSI) and psi / argmax.
__device__ int lp_direction(const LPView& V, const double* x, const double* y, const double* s,
                            const double* rd, double* lds, double* shv, long long* shi,
                            int* s_flag, double* psi_out, long long* arg_out) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = V.m, n = V.n;
  for (int j = tid; j < n; j += 256) {
    const double dj = x[j] / s[j];
    V.d[j] = dj;
    V.w[j] = dj * rd[j];
  }
  __syncthreads();
  for (int i = wv; i < m; i += 4) {
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc += V.A[(long)i * n + j] * V.w[j];
    acc = wsum(acc);
    if (lane == 0) V.rhs[i] = V.b[i] + acc;
  }
  wg_syrk(m, n, V.A, n, V.d, V.M, V.ldm, false, lds);
  double minp;
  const int fail = wg_potrf(m, V.M, V.ldm, lds, &minp);
  if (fail >= 0) {
    *psi_out = NAN;
    *arg_out = -1;
    return LP_ERR_BREAKDOWN;
  }
  wg_trsv_fwd(m, V.M, V.ldm, V.rhs, V.z, lds);
  wg_trsv_bwd(m, V.M, V.ldm, V.z, V.dy, lds);
  double best = -INFINITY;
  long long bi = LLONG_MAX;
  int nz = 0, nf = 0;
  for (int j = tid; j < n; j += 256) {
    double g1 = 0.0, g2 = 0.0;
    for (int i = 0; i < m; ++i) {
      const double av = V.A[(long)i * n + j];
      g1 += av * V.dy[i];
      g2 += av * y[i];
    }
    V.g[j] = g1;
    V.gy[j] = g2;
    const double dsj = rd[j] - g1;
    const double dxj = -x[j] - V.d[j] * dsj;
    V.ds[j] = dsj;
    V.dx[j] = dxj;
    const double u = -dxj / x[j], v = -dsj / s[j];
    nz |= (dxj != 0.0) | (dsj != 0.0);
    nf |= !isfinite(u) | !isfinite(v);
    amerge(best, bi, u, j);
    amerge(best, bi, v, n + j);
  }
  for (int i = tid; i < m; i += 256) nz |= (V.dy[i] != 0.0);
  if (tid == 0) *s_flag = 0;
  __syncthreads();
  if (nz) atomicOr(s_flag, 1);
  if (nf) atomicOr(s_flag, 2);
  bargmax(best, bi, shv, shi);
  const int flags = *s_flag;
  __syncthreads();
  *psi_out = best;
  *arg_out = bi;
  if (!(flags & 1)) return LP_OPTIMAL_ZERO_DIR;
  if ((flags & 2) || !(best > 0) || !isfinite(best)) return LP_ERR_NONPOS_PSI;
  return LP_OK;
}

// Take the next LP from the queue (whole workgroup); -1 when empty.
__device__ inline int next_lp(const BatchArgs& a, int* s_idx) {
  if (threadIdx.x == 0) *s_idx = atomicAdd(a.queue, 1);
  __syncthreads();
  const int idx = *s_idx;
  __syncthreads();
  return idx < a.count ? a.order[idx] : -1;
}

#define PDAS_BATCH_SHARED                                                               \
  __shared__ double lds[2 * 2 * BT * BKC + 2 * BT + BT * (BT + 1) + BT];                \
  __shared__ double sh[4];                                                              \
  __shared__ double shv[4];                                                             \
  __shared__ long long shi[4];                                                          \
  __shared__ int s_idx, s_flag

// One iteration of every still-active LP of the batch.
__global__ __launch_bounds__(256) void k_batch_iter(BatchArgs a) {
  PDAS_BATCH_SHARED;
  const int tid = threadIdx.x;
  for (;;) {
    const int lp = next_lp(a, &s_idx);
    if (lp < 0) break;
    const BatchLP P = a.lps[lp];
    BatchState* S = a.state + lp;
    if (S->status != LP_OK) continue;
    const int m = P.m, n = P.n;
    const int cur = S->cur, nxt = cur ^ 1;
    if (S->gap < a.tol || S->iters >= a.max_iter) {
      __syncthreads();
      if (tid == 0) S->status = (S->gap < a.tol) ? LP_CONVERGED : LP_MAX_ITER;
      continue;
    }
    const LPView V = lp_view(a, P);
    const double* x = a.x[cur] + P.vn;
    const double* y = a.y[cur] + P.vm;
    const double* s = a.s[cur] + P.vn;
    const double* rd = a.rd[cur] + P.vn;
    // tape: start iterate and dual residual of this step
    if (a.tape && S->iters < a.tape_cap) {
      double* row = a.tape + P.tape_off + (long)S->iters * (3 * n + m);
      for (int j = tid; j < n; j += 256) {
        row[j] = x[j];
        row[n + m + j] = s[j];
        row[2 * n + m + j] = rd[j];
      }
      for (int i = tid; i < m; i += 256) row[n + i] = y[i];
    }
    double psi;
    long long bi;
    const int st = lp_direction(V, x, y, s, rd, lds, shv, shi, &s_flag, &psi, &bi);
    if (st != LP_OK) {
      if (tid == 0) {
        S->status = st;
        S->last_psi = psi;
      }
      __syncthreads();
      continue;
    }
    double* xn = a.x[nxt] + P.vn;
    double* yn = a.y[nxt] + P.vm;
    double* sn = a.s[nxt] + P.vn;
    double* rdn = a.rd[nxt] + P.vn;
    const double aeff = (psi == 1.0) ? 1.0 : a.alpha;
    const double t = aeff / psi;
    double gp = 0.0;
    int lost = 0;
    for (int j = tid; j < n; j += 256) {
      const double xv = x[j] + t * V.dx[j];
      const double sv = s[j] + t * V.ds[j];
      xn[j] = xv;
      sn[j] = sv;
      rdn[j] = V.c[j] - (V.gy[j] + t * V.g[j]) - sv;
      gp += xv * sv;
      lost |= !(xv > 0) | !(sv > 0);
    }
    for (int i = tid; i < m; i += 256) yn[i] = y[i] + t * V.dy[i];
    if (tid == 0) s_flag = 0;
    __syncthreads();
    if (lost) atomicOr(&s_flag, 1);
    const double gap = bsum(gp, sh);
    const int lostf = s_flag;
    if (tid == 0) {
      S->last_psi = psi;
      S->last_t = t;
      S->last_argmax = bi;
      if (psi == 1.0) {
        S->status = LP_OPTIMAL_PSI1;
        S->cur = nxt;
        S->gap = gap;
        S->iters += 1;
      } else if (lostf) {
        S->status = LP_ERR_LOST_INTERIOR;
      } else {
        S->cur = nxt;
        S->gap = gap;
        S->iters += 1;
        atomicAdd(a.active, 1);
      }
    }
    __syncthreads();
  }
}

// Reverse of step k for every LP that took at least k + 1 recorded steps:
// the step is recomputed from its tape row, then the chain rule runs back
// through it (same order as the single-LP reverse sweep).  Abar (packed like
// A) accumulates three outer products per step.
__global__ __launch_bounds__(256) void k_batch_backward(BatchArgs a, BatchAdj g, int k) {
  PDAS_BATCH_SHARED;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (;;) {
    const int lp = next_lp(a, &s_idx);
    if (lp < 0) break;
    const BatchLP P = a.lps[lp];
    const BatchState* S = a.state + lp;
    if (k >= S->iters || k >= a.tape_cap) continue;
    const int m = P.m, n = P.n;
    const LPView V = lp_view(a, P);
    const double* row = a.tape + P.tape_off + (long)k * (3 * n + m);
    const double* x = row;
    const double* y = row + n;
    const double* s = row + n + m;
    const double* rd = row + 2 * n + m;
    double psi;
    long long J;
    const int st = lp_direction(V, x, y, s, rd, lds, shv, shi, &s_flag, &psi, &J);
    if (st != LP_OK) {
      if (tid == 0) atomicOr(g.err, 1);
      __syncthreads();
      continue;
    }
    double* xb = g.xb + P.vn;
    double* yb = g.yb + P.vm;
    double* sb = g.sb + P.vn;
    double* dsb = g.dsb + P.vn;
    double* db = g.db + P.vn;
    double* dyb = g.dyb + P.vm;
    double* lam = g.lam + P.vm;
    double* hv = g.h + P.vn;
    double* rdb = g.rdb + P.vn;
    double* bb = g.bbar + P.vm;
    double* cb = g.cbar + P.vn;
    // tbar = xbar.dx + ybar.dy + sbar.ds
    double tp = 0.0;
    for (int j = tid; j < n; j += 256) tp += xb[j] * V.dx[j] + sb[j] * V.ds[j];
    for (int i = tid; i < m; i += 256) tp += yb[i] * V.dy[i];
    const double tbar = bsum(tp, sh);
    const double aeff = (psi == 1.0) ? 1.0 : a.alpha;
    const double t = aeff / psi;
    const double psib = -aeff * tbar / (psi * psi);
    for (int j = tid; j < n; j += 256) {
      double dxb = t * xb[j];
      double dsbj = t * sb[j];
      double xbj = xb[j], sbj = sb[j];
      if (J == j) {
        dxb += -psib / x[j];
        xbj += psib * V.dx[j] / (x[j] * x[j]);
      } else if (J == n + j) {
        dsbj += -psib / s[j];
        sbj += psib * V.ds[j] / (s[j] * s[j]);
      }
      xbj -= dxb;
      db[j] = -dxb * V.ds[j];
      dsbj -= V.d[j] * dxb;
      xb[j] = xbj;
      sb[j] = sbj;
      dsb[j] = dsbj;
    }
    __syncthreads();
    // dybar = t ybar - A dsbar
    for (int i = wv; i < m; i += 4) {
      double acc = 0.0;
      for (int j = lane; j < n; j += 64) acc += V.A[(long)i * n + j] * dsb[j];
      acc = wsum(acc);
      if (lane == 0) dyb[i] = t * yb[i] - acc;
    }
    __syncthreads();
    // lambda = M^-1 dybar with the recomputed factor
    wg_trsv_fwd(m, V.M, V.ldm, dyb, V.z, lds);
    wg_trsv_bwd(m, V.M, V.ldm, V.z, lam, lds);
    // h = A^T lambda, then d, rhs and r_d in reverse
    for (int j = tid; j < n; j += 256) {
      double h = 0.0;
      for (int i = 0; i < m; ++i) h += V.A[(long)i * n + j] * lam[i];
      hv[j] = h;
      double dbj = db[j];
      dbj -= h * V.g[j];
      dbj += rd[j] * h;
      const double rdbj = dsb[j] + V.d[j] * h;
      xb[j] += dbj / s[j];
      sb[j] = sb[j] - dbj * x[j] / (s[j] * s[j]) - rdbj;
      cb[j] += rdbj;
      rdb[j] = rdbj;
    }
    for (int i = tid; i < m; i += 256) bb[i] += lam[i];
    __syncthreads();
    // ybar -= A rdbar
    for (int i = wv; i < m; i += 4) {
      double acc = 0.0;
      for (int j = lane; j < n; j += 64) acc += V.A[(long)i * n + j] * rdb[j];
      acc = wsum(acc);
      if (lane == 0) yb[i] -= acc;
    }
    // Abar += dy v1^T + lambda v2^T + y v3^T
    if (g.Abar) {
      double* Ab = g.Abar + P.a_off;
      for (int i = wv; i < m; i += 4) {
        const double u1 = V.dy[i], u2 = lam[i], u3 = y[i];
        for (int j = lane; j < n; j += 64) {
          const double v1 = -dsb[j] - hv[j] * V.d[j];
          const double v2 = V.d[j] * rd[j] - V.g[j] * V.d[j];
          const double v3 = -rdb[j];
          Ab[(long)i * n + j] += u1 * v1 + u2 * v2 + u3 * v3;
        }
      }
    }
    __syncthreads();
  }
}

// Reset the queue and active counters before each iteration (a kernel, so
// the reset is a plain node of a captured graph).
__global__ void k_batch_reset(int* queue, int* active) {
  if (threadIdx.x == 0) {
    *queue = 0;
    *active = 0;
  }
}

// x^T s of every LP (setup).
__global__ __launch_bounds__(256) void k_batch_gap(int count, const BatchLP* lps,
                                                   BatchState* state, const double* x,
                                                   const double* s) {
  __shared__ double sh[4];
  const int lp = blockIdx.x;
  if (lp >= count) return;
  const BatchLP P = lps[lp];
  double v = 0.0;
  for (int j = threadIdx.x; j < P.n; j += 256) v += x[P.vn + j] * s[P.vn + j];
  const double gp = bsum(v, sh);
  if (threadIdx.x == 0) state[lp].gap = gp;
}

// r_d = c - A^T y - s of every LP (setup).
__global__ __launch_bounds__(256) void k_batch_rd(int count, const BatchLP* lps, const double* Ap,
                                                  const double* c, const double* y,
                                                  const double* s, double* rd) {
  const int lp = blockIdx.x;
  if (lp >= count) return;
  const BatchLP P = lps[lp];
  const double* A = Ap + P.a_off;
  for (int j = threadIdx.x; j < P.n; j += 256) {
    double acc = 0.0;
    for (int i = 0; i < P.m; ++i) acc += A[(long)i * P.n + j] * y[P.vm + i];
    rd[P.vn + j] = c[P.vn + j] - acc - s[P.vn + j];
  }
}

void launch_batch_iter(hipStream_t st, const BatchArgs& args, int grid) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, args.queue, args.active);
  hipLaunchKernelGGL(k_batch_iter, dim3(grid), dim3(256), 0, st, args);
}

void launch_batch_backward(hipStream_t st, const BatchArgs& args, const BatchAdj& adj, int k,
                           int grid) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, args.queue, args.active);
  hipLaunchKernelGGL(k_batch_backward, dim3(grid), dim3(256), 0, st, args, adj, k);
}

void launch_batch_setup(hipStream_t st, int count, const BatchLP* lps, BatchState* state,
                        const double* Ap, const double* c, const double* x, const double* y,
                        const double* s, double* rd) {
  hipLaunchKernelGGL(k_batch_rd, dim3(count), dim3(256), 0, st, count, lps, Ap, c, y, s, rd);
  hipLaunchKernelGGL(k_batch_gap, dim3(count), dim3(256), 0, st, count, lps, state, x, s);
}

}  // namespace pdas
