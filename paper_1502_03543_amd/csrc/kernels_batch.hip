// Batched Primal-Dual Affine Scaling: many independent LPs of their own
// shapes (m_i, n_i), each advanced by the Section 3 iteration (Section 5
// normal equations, Cholesky of Section 5.1).
//
// One iteration of the whole batch is a fixed sequence of launches whose
// grids depend only on the batch (count, largest m and n), so the host
// captures it once into a hipGraph and replays it:
//   k_bbegin        per LP: stop tests, tape row, d = x/s, w = d o r_d
//   k_bsyrk_normal16 per LP and lower 32- or 64-tile: M = A D A^T on the
//                   FP64 matrix cores (16 x 16 x 4 blocks, an LP's tiles on
//                   one XCD); its diagonal tiles also form rhs = b + A w.
//                   128-tiles run the stream-K tile routine, and k_brhs
//                   (wavefront per row) forms rhs beside them and in the
//                   mixed-precision iterations
//   per panel p:    k_bpotrf_panel (the single-LP panel routine), then
//                   k_bsyrk_trailing (the tile routine in subtract mode);
//                   k_bdiag_to_m puts the diagonal blocks into M at the end
//   k_btrsv         per LP: L z = rhs, L^T dy = z (64-row blocks, readlane)
//   k_bdir          per LP and 256-column slice: g = A^T dy, g_y = A^T y,
//                   ds, dx, the slice's ratio-test maximiser
//   k_bdir_fin      per LP: merged maximiser psi, statuses
//   k_bstep         per LP: step, next r_d, gap, statuses
// The reverse sweep recomputes step k from its tape row with the same
// launches (k_bbegin reads the tape instead of the iterate) and ends with the
// five reverse launches k_badj_t, k_badj_dyb, k_badj_solve, k_badj_h and
// k_badj_yb in place of k_bstep; k_babar forms Abar once after the sweep.
// LPs that stopped skip every launch (a flag per LP), so a replay costs
// nothing for them.
#include <climits>
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

constexpr int BT = 64;  // triangular-solve block

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

// The 64 x 64 diagonal block at (i0, i0) of L (rows < nr kept, identity
// beyond, upper part zero) into an LDS block of row length BT + 1.
// diag_first: by the whole workgroup; diag_next: by wavefronts 1..3 while
// wavefront 0 solves the current block from the other LDS block.  Either
// way all loads of a thread are issued before its first LDS store.
constexpr int kLdBlk = BT * (BT + 1);

// A zero the compiler cannot see through: index arithmetic offset by it is
// redone at each use instead of being hoisted out of the block loop, where
// its per-element values would stay live in registers across every block.
__device__ inline int opaque_zero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}

template <int NT>
__device__ __forceinline__ void diag_stage(const double* L, long ld, int i0, int nr, int t0,
                                           double* Ld) {
  constexpr int Q = (BT * BT + NT - 1) / NT;
  const int t = t0 + opaque_zero();
  double v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = t + NT * q, ii = e / BT, k = e % BT;
    v[q] = (e < BT * BT && ii < nr && k <= ii) ? L[(long)(i0 + ii) * ld + i0 + k]
                                                : ((ii == k) ? 1.0 : 0.0);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = t + NT * q;
    if (e < BT * BT) Ld[(e / BT) * (BT + 1) + e % BT] = v[q];
  }
}
__device__ __forceinline__ void diag_first(const double* L, long ld, int i0, int nr, int tid,
                                           double* Ld) {
  diag_stage<256>(L, ld, i0, nr, tid, Ld);
}
__device__ __forceinline__ void diag_next(const double* L, long ld, int i0, int nr, int tid,
                                          double* Ld) {
  diag_stage<192>(L, ld, i0, nr, tid - 64, Ld);
}

// LDS of the workgroup solves (doubles): partial sums, two diagonal blocks
constexpr int kTrsvLds = 4 * BT + 2 * kLdBlk;

// z = L^-1 r (forward) into out; L row-major lower with ld.  One workgroup:
// per 64-row block, all threads form the off-diagonal product, then wave 0
// solves the diagonal block (staged in LDS by the other waves during the
// previous block's solve) with readlane broadcasts.
__device__ __forceinline__ void wg_trsv_fwd(int m, const double* L, long ld, const double* r,
                                            double* out, double* lds) {
  double* sacc = lds;  // [64]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i0 = 0; i0 < m; i0 += BT) {
    const int rows = min(BT, m - i0);
    double* Ld = lds + 4 * BT + ((i0 / BT) & 1) * kLdBlk;
    if (i0 == 0) diag_first(L, ld, i0, rows, tid, Ld);
    // wave wv: rows 16 wv .. 16 wv + 15, lanes over columns 0..i0-1; the
    // sixteen rows' loads of a column group are issued together
    {
      constexpr int RPW = BT / 4;
      const double* Lw = L + (long)(i0 + RPW * wv) * ld;
      const int nr = min(RPW, rows - RPW * wv);
      double acc[RPW];
#pragma unroll
      for (int q = 0; q < RPW; ++q) acc[q] = 0.0;
      if (nr > 0) {
        // rows past the last are read as the last row (in the matrix, so
        // every load is issued without a branch) and weighted by zero
        for (int c = lane; c < i0; c += 64) {
          const double oc = out[c];
          double lv[RPW];
#pragma unroll
          for (int q = 0; q < RPW; ++q) lv[q] = Lw[(long)min(q, nr - 1) * ld + c];
#pragma unroll
          for (int q = 0; q < RPW; ++q) acc[q] += lv[q] * (q < nr ? oc : 0.0);
        }
      }
      // the sixteen lane sums reduced together: each butterfly level hands
      // half of the remaining rows to the partner lane, so after four
      // levels lane l holds row (l / 4) % 16 summed over its 16 lanes, and
      // two more levels finish the sums over all 64
#pragma unroll
      for (int h = RPW / 2, o = 32; h >= 1; h >>= 1, o >>= 1) {
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int q = 0; q < h; ++q) {
          const double keep = up ? acc[q + h] : acc[q];
          const double send = up ? acc[q] : acc[q + h];
          acc[q] = keep + __shfl_xor(send, o, 64);
        }
      }
      double v = acc[0];
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 1, 64);
      if ((lane & 3) == 0) sacc[RPW * wv + ((lane >> 2) & 15)] = v;
    }
    __syncthreads();
    // wavefronts 1..3 stage the next diagonal block while wavefront 0 solves
    if (wv > 0 && i0 + BT < m)
      diag_next(L, ld, i0 + BT, min(BT, m - i0 - BT), tid, lds + 4 * BT + ((i0 / BT + 1) & 1) * kLdBlk);
    if (wv == 0) {
      // each row scaled by its pivot's reciprocal, so that step j is one
      // broadcast and one fused multiply-add: z_j is row j's value itself,
      // and the scaled multipliers (zero where row i does not take step j)
      // are formed beside the chain
      const double dl = 1.0 / Ld[lane * (BT + 1) + lane];
      double val = ((lane < rows) ? (r[i0 + lane] - sacc[lane]) : 0.0) * dl;
      double mine = 0.0;
#pragma unroll 4
      for (int j = 0; j < BT; ++j) {
        // (read by every lane, zeroed through the scale: no branch)
        const double lij = Ld[lane * (BT + 1) + j] * (lane > j ? dl : 0.0);
        const double zj = rl(val, j);
        mine = lane == j ? zj : mine;
        val = fma(-lij, zj, val);
      }
      if (lane < rows) out[i0 + lane] = mine;
    }
    __syncthreads();
  }
}

// y = L^-T z into out.
__device__ __forceinline__ void wg_trsv_bwd(int m, const double* L, long ld, const double* z,
                                            double* out, double* lds) {
  double* sacc = lds;  // [4][64]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nblk = (m + BT - 1) / BT;
  for (int rb = nblk - 1; rb >= 0; --rb) {
    const int c0 = rb * BT, cols = min(BT, m - c0);
    double* Ld = lds + 4 * BT + ((nblk - 1 - rb) & 1) * kLdBlk;
    if (rb == nblk - 1) diag_first(L, ld, c0, cols, tid, Ld);
    double acc = 0.0;
    if (lane < cols) {
#pragma unroll 8
      for (int i = c0 + BT + wv; i < m; i += 4) acc += L[(long)i * ld + c0 + lane] * out[i];
    }
    sacc[wv * BT + lane] = acc;
    __syncthreads();
    // wavefronts 1..3 stage the next diagonal block while wavefront 0 solves
    if (wv > 0 && rb > 0) diag_next(L, ld, c0 - BT, BT, tid, lds + 4 * BT + ((nblk - rb) & 1) * kLdBlk);
    if (wv == 0) {
      // scaled as in the forward solve: one broadcast and one fused
      // multiply-add per step
      const double dl = 1.0 / Ld[lane * (BT + 1) + lane];
      const double tot = ((sacc[lane] + sacc[BT + lane]) + sacc[2 * BT + lane]) + sacc[3 * BT + lane];
      double val = ((lane < cols) ? (z[c0 + lane] - tot) : 0.0) * dl;
      double mine = 0.0;
#pragma unroll 4
      for (int j = BT - 1; j >= 0; --j) {
        const double lji = Ld[j * (BT + 1) + lane] * (lane < j ? dl : 0.0);
        const double yj = rl(val, j);
        mine = lane == j ? yj : mine;
        val = fma(-lji, yj, val);
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

// Source iterate of LP P for this launch sequence: the current iterate
// (k < 0) or the tape row of step k.
__device__ inline void lp_source(const BatchArgs& a, const BatchLP& P, int cur, int k,
                                 const double*& x, const double*& y, const double*& s,
                                 const double*& rd) {
  if (k < 0) {
    x = a.x[cur] + P.vn;
    y = a.y[cur] + P.vm;
    s = a.s[cur] + P.vn;
    rd = a.rd[cur] + P.vn;
  } else {
    const double* row = a.tape + P.tape_off + (long)k * (3 * P.n + P.m);
    x = row;
    y = row + P.n;
    s = row + P.n + P.m;
    rd = row + 2 * P.n + P.m;
  }
}

namespace {

// Stop tests (forward) or the reverse filter (k >= 0); tape row; d and w.
__global__ __launch_bounds__(256) void k_bbegin(BatchArgs a, int k) {
  __shared__ int s_go, s_cur, s_iters;
  const int lp = blockIdx.x;
  const BatchLP P = a.lps[lp];
  BatchState* S = a.state + lp;
  if (threadIdx.x == 0) {
    int go = 0;
    if (k < 0) {
      if (S->status == LP_OK) {
        if (S->gap < a.tol) S->status = LP_CONVERGED;
        else if (S->iters >= a.max_iter) S->status = LP_MAX_ITER;
        else go = 1;
      }
    } else {
      go = (k < S->iters && k < a.tape_cap) ? 1 : 0;
    }
    a.go[lp] = go;
    a.fail[lp] = INT_MAX;
    a.minp[lp] = 0x7ff0000000000000ull;  // +inf
    s_go = go;
    s_cur = S->cur;
    s_iters = S->iters;
  }
  __syncthreads();
  if (!s_go) return;
  const double *x, *y, *s, *rd;
  lp_source(a, P, s_cur, k, x, y, s, rd);
  const int n = P.n, m = P.m;
  if (k < 0 && a.tape && s_iters < a.tape_cap) {
    double* row = a.tape + P.tape_off + (long)s_iters * (3 * n + m);
    for (int j = threadIdx.x; j < n; j += 256) {
      row[j] = x[j];
      row[n + m + j] = s[j];
      row[2 * n + m + j] = rd[j];
    }
    for (int i = threadIdx.x; i < m; i += 256) row[n + i] = y[i];
  }
  double* d = a.d + P.vn;
  double* w = a.w + P.vn;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double dj = x[j] / s[j];
    d[j] = dj;
    w[j] = dj * rd[j];
  }
}

// rhs = b + A w: one wavefront per row, four rows per workgroup.
__global__ __launch_bounds__(256) void k_brhs(BatchArgs a) {
  const int lp = blockIdx.y;
  if (!a.go[lp]) return;
  const BatchLP P = a.lps[lp];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= P.m) return;
  const double* Ai = a.A + P.a_off + (long)i * P.n;
  const double* w = a.w + P.vn;
  double acc = 0.0;
  for (int j = lane; j < P.n; j += 64) acc += Ai[j] * w[j];
  acc = wsum(acc);
  if (lane == 0) a.rhs[P.vm + i] = a.b[P.vm + i] + acc;
}

// Breakdown check, then L z = rhs and L^T dy = z.
// (go_main, when given, is the stepping flag to clear on a breakdown when
// a.go is a narrower mask: the FP64 factor of a mixed-precision batch.)
__global__ __launch_bounds__(256) void k_btrsv(BatchArgs a, int k, int* err, int* go_main) {
  __shared__ double lds[kTrsvLds];
  const int lp = blockIdx.x;
  if (!a.go[lp]) return;
  const BatchLP P = a.lps[lp];
  if (a.fail[lp] != INT_MAX) {
    if (threadIdx.x == 0) {
      if (k < 0) {
        a.state[lp].status = LP_ERR_BREAKDOWN;
        a.state[lp].last_psi = NAN;
      } else {
        atomicOr(err, 1);
      }
      a.go[lp] = 0;
      if (go_main) go_main[lp] = 0;
    }
    return;
  }
  const double* M = a.M + P.M_off;
  wg_trsv_fwd(P.m, M, P.ldm, a.rhs + P.vm, a.z + P.vm, lds);
  wg_trsv_bwd(P.m, M, P.ldm, a.z + P.vm, a.dy + P.vm, lds);
}

// g = A^T dy, g_y = A^T y, ds = r_d - g, dx = -x - d o ds, psi and its first
// maximiser (x block before s block); zero and non-finite directions.  One
// workgroup per LP and slice of 256 columns (a thread per column), so a large
// LP's pass over A is spread over several compute units; each slice leaves
// its maximiser and flags, k_bdir_fin merges them per LP.
constexpr int kDirStage = 1024;  // dy and y entries staged in LDS per LP

__global__ __launch_bounds__(256) void k_bdir(BatchArgs a, int k) {
  __shared__ double shv[4];
  __shared__ long long shi[4];
  __shared__ int s_flag, s_cur;
  __shared__ double sdy[kDirStage], sy[kDirStage];
  const int lp = blockIdx.y, sl = blockIdx.x;
  if (!a.go[lp]) return;
  const BatchLP P = a.lps[lp];
  const int m = P.m, n = P.n;
  if (sl * 256 >= n) return;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_flag = 0;
    s_cur = a.state[lp].cur;
  }
  __syncthreads();
  const LPView V = lp_view(a, P);
  const double *x, *y, *s, *rd;
  lp_source(a, P, s_cur, k, x, y, s, rd);
  double best = -INFINITY;
  long long bi = LLONG_MAX;
  int nz = 0, nf = 0;
  const int ms = min(m, kDirStage);
  for (int i = tid; i < ms; i += 256) {
    sdy[i] = V.dy[i];
    sy[i] = y[i];
  }
  __syncthreads();
  const int j = sl * 256 + tid;
  if (j < n) {
    // sums in row order; the column's A entries are loaded eight rows ahead
    // so the loads overlap instead of following one another
    double g1 = 0.0, g2 = 0.0;
    const double* acol = V.A + j;
    int i = 0;
    for (; i + 8 <= ms; i += 8) {
      double av[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) av[u] = acol[(long)(i + u) * n];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        g1 += av[u] * sdy[i + u];
        g2 += av[u] * sy[i + u];
      }
    }
    for (; i < ms; ++i) {
      const double av = acol[(long)i * n];
      g1 += av * sdy[i];
      g2 += av * sy[i];
    }
    for (; i < m; ++i) {
      const double av = acol[(long)i * n];
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
  if (sl == 0)
    for (int i = tid; i < m; i += 256) nz |= (V.dy[i] != 0.0);
  if (nz) atomicOr(&s_flag, 1);
  if (nf) atomicOr(&s_flag, 2);
  bargmax(best, bi, shv, shi);
  if (tid != 0) return;
  const long o = (long)lp * a.nslice + sl;
  a.dpv[o] = best;
  a.dpi[o] = bi;
  a.dpf[o] = s_flag;
}

// Per LP (a thread each): merge the slices' maximisers (largest value, then
// smallest index, so the order of the merge does not matter) and flags into
// psi, its argmax and the LP's status.
__global__ __launch_bounds__(256) void k_bdir_fin(BatchArgs a, int k, int* err) {
  const int lp = blockIdx.x * 256 + threadIdx.x;
  if (lp >= a.count || !a.go[lp]) return;
  const int ns = (a.lps[lp].n + 255) / 256;
  const long o = (long)lp * a.nslice;
  double best = -INFINITY;
  long long bi = LLONG_MAX;
  int flags = 0;
  for (int q = 0; q < ns; ++q) {
    amerge(best, bi, a.dpv[o + q], a.dpi[o + q]);
    flags |= a.dpf[o + q];
  }
  a.psi[lp] = best;
  a.arg[lp] = bi;
  int st = LP_OK;
  if (!(flags & 1)) st = LP_OPTIMAL_ZERO_DIR;
  else if ((flags & 2) || !(best > 0) || !isfinite(best)) st = LP_ERR_NONPOS_PSI;
  if (st != LP_OK) {
    if (k < 0) {
      a.state[lp].status = st;
      a.state[lp].last_psi = best;
    } else {
      atomicOr(err, 1);
    }
    a.go[lp] = 0;
  }
}

// The step: alpha_eff = 1 when psi == 1, t = alpha_eff / psi, new iterate into
// the other buffer, next r_d, gap; statuses.
__global__ __launch_bounds__(256) void k_bstep(BatchArgs a) {
  __shared__ double sh[4];
  __shared__ int s_flag, s_cur;
  const int lp = blockIdx.x;
  if (!a.go[lp]) return;
  const int tid = threadIdx.x;
  const BatchLP P = a.lps[lp];
  BatchState* S = a.state + lp;
  if (tid == 0) {
    s_flag = 0;
    s_cur = S->cur;
  }
  __syncthreads();
  const int cur = s_cur, nxt = cur ^ 1;
  const LPView V = lp_view(a, P);
  const double *x, *y, *s, *rd;
  lp_source(a, P, cur, -1, x, y, s, rd);
  const int m = P.m, n = P.n;
  double* xn = a.x[nxt] + P.vn;
  double* yn = a.y[nxt] + P.vm;
  double* sn = a.s[nxt] + P.vn;
  double* rdn = a.rd[nxt] + P.vn;
  const double psi = a.psi[lp];
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
  if (lost) atomicOr(&s_flag, 1);
  const double gap = bsum(gp, sh);
  const int lostf = s_flag;
  if (tid == 0) {
    S->last_psi = psi;
    S->last_t = t;
    S->last_argmax = a.arg[lp];
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
}

// Reverse of the recomputed step k of LP blockIdx.x (same order as the
// single-LP reverse sweep).  Abar (packed like A) accumulates three outer
// products per step.
// The reverse step runs as five launches: the per-LP scalar part and the
// triangular solves take one workgroup per LP, the three products with A
// (A dsbar, A^T lambda, A rdbar) one wavefront per row or one thread per
// column across all LPs, each sum in the same order as a single workgroup
// would take it.
struct AdjPtrs {
  double *xb, *yb, *sb, *dsb, *db, *dyb, *lam, *hv, *rdb, *bb, *cb;
};
__device__ inline AdjPtrs adj_ptrs(const BatchAdj& g, const BatchLP& P) {
  return AdjPtrs{g.xb + P.vn,   g.yb + P.vm, g.sb + P.vn,  g.dsb + P.vn,
                 g.db + P.vn,   g.dyb + P.vm, g.lam + P.vm, g.h + P.vn,
                 g.rdb + P.vn,  g.bbar + P.vm, g.cbar + P.vn};
}
__device__ inline double adj_t(const BatchArgs& a, int lp) {
  const double psi = a.psi[lp];
  const double aeff = (psi == 1.0) ? 1.0 : a.alpha;
  return aeff / psi;
}

// 1. tbar = xbar.dx + ybar.dy + sbar.ds, the ratio test and the step in
//    reverse (one workgroup per LP)
__global__ __launch_bounds__(256) void k_badj_t(BatchArgs a, BatchAdj g, int k) {
  __shared__ double sh[4];
  const int lp = blockIdx.x;
  if (!a.go[lp]) return;
  const int tid = threadIdx.x;
  const BatchLP P = a.lps[lp];
  const int m = P.m, n = P.n;
  const LPView V = lp_view(a, P);
  const double *x, *y, *s, *rd;
  lp_source(a, P, 0, k, x, y, s, rd);
  const double psi = a.psi[lp];
  const long long J = a.arg[lp];
  const AdjPtrs q = adj_ptrs(g, P);
  double tp = 0.0;
  for (int j = tid; j < n; j += 256) tp += q.xb[j] * V.dx[j] + q.sb[j] * V.ds[j];
  for (int i = tid; i < m; i += 256) tp += q.yb[i] * V.dy[i];
  const double tbar = bsum(tp, sh);
  const double aeff = (psi == 1.0) ? 1.0 : a.alpha;
  const double t = aeff / psi;
  const double psib = -aeff * tbar / (psi * psi);
  for (int j = tid; j < n; j += 256) {
    double dxb = t * q.xb[j];
    double dsbj = t * q.sb[j];
    double xbj = q.xb[j], sbj = q.sb[j];
    if (J == j) {
      dxb += -psib / x[j];
      xbj += psib * V.dx[j] / (x[j] * x[j]);
    } else if (J == n + j) {
      dsbj += -psib / s[j];
      sbj += psib * V.ds[j] / (s[j] * s[j]);
    }
    xbj -= dxb;
    q.db[j] = -dxb * V.ds[j];
    dsbj -= V.d[j] * dxb;
    q.xb[j] = xbj;
    q.sb[j] = sbj;
    q.dsb[j] = dsbj;
  }
}

// 2. dybar = t ybar - A dsbar: one wavefront per row (blockIdx.x * 4 + wave)
__global__ __launch_bounds__(256) void k_badj_dyb(BatchArgs a, BatchAdj g) {
  const int lp = blockIdx.y;
  if (!a.go[lp]) return;
  const BatchLP P = a.lps[lp];
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= P.m) return;
  const int n = P.n;
  const double* Ai = a.A + P.a_off + (long)i * n;
  const double* dsb = g.dsb + P.vn;
  double acc = 0.0;
#pragma unroll 8
  for (int j = lane; j < n; j += 64) acc += Ai[j] * dsb[j];
  acc = wsum(acc);
  if (lane == 0) g.dyb[P.vm + i] = adj_t(a, lp) * g.yb[P.vm + i] - acc;
}

// 3. lambda = M^-1 dybar with the recomputed factor (one workgroup per LP)
__global__ __launch_bounds__(256) void k_badj_solve(BatchArgs a, BatchAdj g) {
  __shared__ double lds[kTrsvLds];
  const int lp = blockIdx.x;
  if (!a.go[lp]) return;
  const BatchLP P = a.lps[lp];
  const LPView V = lp_view(a, P);
  wg_trsv_fwd(P.m, V.M, V.ldm, g.dyb + P.vm, V.z, lds);
  wg_trsv_bwd(P.m, V.M, V.ldm, V.z, g.lam + P.vm, lds);
}

// 4. h = A^T lambda (one thread per column, rows in order), then d, rhs and
//    r_d in reverse; bbar += lambda; the column vectors of this step's share
//    of Abar (slot k)
__global__ __launch_bounds__(256) void k_badj_h(BatchArgs a, BatchAdj g, int k) {
  const int lp = blockIdx.y;
  if (!a.go[lp]) return;
  const BatchLP P = a.lps[lp];
  const int m = P.m, n = P.n;
  const LPView V = lp_view(a, P);
  const double *x, *y, *s, *rd;
  lp_source(a, P, 0, k, x, y, s, rd);
  const AdjPtrs q = adj_ptrs(g, P);
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < m; i += 256) q.bb[i] += q.lam[i];
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double h = 0.0;
#pragma unroll 16
  for (int i = 0; i < m; ++i) h += V.A[(long)i * n + j] * q.lam[i];
  q.hv[j] = h;
  double dbj = q.db[j];
  dbj -= h * V.g[j];
  dbj += rd[j] * h;
  const double rdbj = q.dsb[j] + V.d[j] * h;
  q.xb[j] += dbj / s[j];
  q.sb[j] = q.sb[j] - dbj * x[j] / (s[j] * s[j]) - rdbj;
  q.cb[j] += rdbj;
  q.rdb[j] = rdbj;
  // this step's share of Abar, dy v1^T + lambda v2^T + y v3^T: the six
  // vectors are kept (slot k) and the products formed once after the sweep
  // (k_babar), instead of reading and writing all of Abar every step
  if (g.Abar) {
    double* W = g.vfac + (long)k * 3 * g.sn + P.vn;
    W[j] = -q.dsb[j] - h * V.d[j];
    W[g.sn + j] = V.d[j] * rd[j] - V.g[j] * V.d[j];
    W[2 * g.sn + j] = -rdbj;
  }
}

// 5. ybar -= A rdbar (one wavefront per row); the row vectors of the step's
//    share of Abar
__global__ __launch_bounds__(256) void k_badj_yb(BatchArgs a, BatchAdj g, int k) {
  const int lp = blockIdx.y;
  if (!a.go[lp]) return;
  const BatchLP P = a.lps[lp];
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= P.m) return;
  const int n = P.n;
  const double* Ai = a.A + P.a_off + (long)i * n;
  const double* rdb = g.rdb + P.vn;
  double acc = 0.0;
#pragma unroll 8
  for (int j = lane; j < n; j += 64) acc += Ai[j] * rdb[j];
  acc = wsum(acc);
  if (lane == 0) {
    g.yb[P.vm + i] -= acc;
    if (g.Abar) {
      const double *x, *y, *s, *rd;
      lp_source(a, P, 0, k, x, y, s, rd);
      double* U = g.ufac + (long)k * 3 * g.sm + P.vm;
      U[i] = a.dy[P.vm + i];
      U[g.sm + i] = g.lam[P.vm + i];
      U[2 * g.sm + i] = y[i];
    }
  }
}

// Abar of LP blockIdx.y, 64 x 64 tile blockIdx.x: the sum over the steps the
// sweep reversed (last first, as it ran) of dy v1^T + lambda v2^T + y v3^T,
// each step's three products added as one term.  Thread t: column t % 64,
// rows t / 64 + 4 e.
__global__ __launch_bounds__(256) void k_babar(const BatchLP* __restrict__ lps,
                                               const BatchState* __restrict__ st, BatchAdj g,
                                               int tape_cap, double* __restrict__ Abar) {
  const int lp = blockIdx.y;
  const BatchLP P = lps[lp];
  const int tn = (P.n + 63) / 64, tm = (P.m + 63) / 64;
  const int t = blockIdx.x;
  if (t >= tm * tn) return;
  const int r0 = (t / tn) * 64, j = (t % tn) * 64 + (threadIdx.x & 63), rw = threadIdx.x >> 6;
  if (j >= P.n) return;
  const int nk = min(st[lp].iters, tape_cap);
  double acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;
  for (int k = nk - 1; k >= 0; --k) {
    const double* U = g.ufac + (long)k * 3 * g.sm + P.vm;
    const double* W = g.vfac + (long)k * 3 * g.sn + P.vn;
    const double v1 = W[j], v2 = W[g.sn + j], v3 = W[2 * g.sn + j];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = min(r0 + rw + 4 * e, P.m - 1);
      acc[e] += U[i] * v1 + U[g.sm + i] * v2 + U[2 * g.sm + i] * v3;
    }
  }
  double* Ab = Abar + P.a_off;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int i = r0 + rw + 4 * e;
    if (i < P.m) Ab[(long)i * P.n + j] = acc[e];
  }
}

// Clear the count of LPs still iterating (a kernel, so it is a plain node of
// a captured graph).
__global__ void k_bclear(int* active) {
  if (threadIdx.x == 0) *active = 0;
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

// ---------------------------------------------------------------------------
// Mixed precision (lp_options.precision == LP_PREC_MIXED), per LP as in the
// single-LP solver: an FP32 normal matrix (sqrt(d) on both operands) and
// FP32 factor, widened to FP64 for the solves, then up to refine_max FP64
// corrections on the matrix-free residual r = rhs - A (d o (A^T dy)); an
// LP whose FP32 pivot fails, whose corrections stall (a correction not
// below half the previous one) or that has not converged after refine_max
// corrections takes the FP64 factor in the same iteration and keeps it.
// Convergence: ||delta||_inf / ||dy||_inf <= tol, or, once the corrections
// contract by q < 1/2, ||delta|| q / (1 - q) / ||dy|| <= tol.
enum { kRefRun = 0, kRefOk = 1, kRefFail = 2, kRefNone = 3 };

// A32 with rows padded to n4 (zeros beyond n): one workgroup per row group.
__global__ __launch_bounds__(256) void k_bmix_a32(const BatchLP* __restrict__ lps,
                                                   const double* __restrict__ A, float* A32) {
  const int lp = blockIdx.y;
  const BatchLP P = lps[lp];
  const int i = blockIdx.x;
  if (i >= P.m) return;
  const double* src = A + P.a_off + (long)i * P.n;
  float* dst = A32 + P.a32_off + (long)i * P.n4;
  for (int j = threadIdx.x; j < P.n4; j += 256) dst[j] = j < P.n ? (float)src[j] : 0.f;
}

// Which factor each stepping LP takes this iteration; sqrt(d) in FP32.
__global__ __launch_bounds__(256) void k_bmix_begin(BatchArgs a) {
  const int lp = blockIdx.x;
  const BatchLP P = a.lps[lp];
  __shared__ int s_m32;
  if (threadIdx.x == 0) {
    const int go = a.go[lp];
    if (go && a.fp32_mode[lp] && !(a.state[lp].gap >= a.switch_gap)) a.fp32_mode[lp] = 0;
    const int m32 = go && a.fp32_mode[lp];
    a.m32[lp] = m32;
    a.go64[lp] = go && !m32;
    a.refm[lp] = 0;
    a.ref_status[lp] = m32 ? kRefRun : kRefNone;
    a.ref_steps[lp] = 0;
    a.ref_prev[lp] = INFINITY;
    s_m32 = m32;
  }
  __syncthreads();
  if (!s_m32) return;
  const double* d = a.d + P.vn;
  float* sd = a.sd32 + P.vn4;
  for (int j = threadIdx.x; j < P.n4; j += 256) sd[j] = j < P.n ? (float)sqrt(d[j]) : 0.f;
}

// After the FP32 factor: a failed pivot ends the FP32 attempt; otherwise L
// is widened into the FP64 matrix and the first solve gives dy.
__global__ __launch_bounds__(256) void k_bmix_solve0(BatchArgs a) {
  __shared__ double lds[kTrsvLds];
  const int lp = blockIdx.x;
  if (!a.m32[lp]) return;
  const BatchLP P = a.lps[lp];
  if (a.fail[lp] != INT_MAX) {
    if (threadIdx.x == 0) a.ref_status[lp] = kRefFail;
    return;
  }
  const float* L32 = a.M32 + P.m32_off;
  double* M = a.M + P.M_off;
  const int m = P.m;
  for (long e = threadIdx.x; e < (long)m * m; e += 256) {
    const int r = (int)(e / m), c = (int)(e % m);
    if (c <= r) M[(long)r * P.ldm + c] = (double)L32[(long)r * P.ld32 + c];
  }
  __syncthreads();
  wg_trsv_fwd(m, M, P.ldm, a.rhs + P.vm, a.z + P.vm, lds);
  wg_trsv_bwd(m, M, P.ldm, a.z + P.vm, a.dy + P.vm, lds);
  if (threadIdx.x == 0) a.refm[lp] = 1;
}

// v = d o (A^T dy): one workgroup per LP and 256-column slice.
__global__ __launch_bounds__(256) void k_bref_v(BatchArgs a) {
  const int lp = blockIdx.y, sl = blockIdx.x;
  if (!a.refm[lp]) return;
  const BatchLP P = a.lps[lp];
  const int j = sl * 256 + threadIdx.x;
  if (j >= P.n) return;
  const double* acol = a.A + P.a_off + j;
  const double* dy = a.dy + P.vm;
  double g = 0.0;
  int i = 0;
  for (; i + 8 <= P.m; i += 8) {
    double av[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) av[u] = acol[(long)(i + u) * P.n];
#pragma unroll
    for (int u = 0; u < 8; ++u) g += av[u] * dy[i + u];
  }
  for (; i < P.m; ++i) g += acol[(long)i * P.n] * dy[i];
  a.v[P.vn + j] = a.d[P.vn + j] * g;
}

// r = rhs - A v: one wavefront per row, four rows per workgroup.
__global__ __launch_bounds__(256) void k_bref_r(BatchArgs a) {
  const int lp = blockIdx.y;
  if (!a.refm[lp]) return;
  const BatchLP P = a.lps[lp];
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= P.m) return;  // whole wavefronts
  const double* arow = a.A + P.a_off + (long)i * P.n;
  const double* v = a.v + P.vn;
  double acc = 0.0;
  for (int j = lane; j < P.n; j += 64) acc += arow[j] * v[j];
  acc = wsum(acc);
  if (lane == 0) a.r[P.vm + i] = a.rhs[P.vm + i] - acc;
}

// delta = L^-T L^-1 r, dy += delta, then the convergence test.
__global__ __launch_bounds__(256) void k_bref_solve(BatchArgs a) {
  __shared__ double lds[kTrsvLds];
  const int lp = blockIdx.x;
  if (!a.refm[lp]) return;
  const BatchLP P = a.lps[lp];
  const double* M = a.M + P.M_off;
  double* delta = a.delta + P.vm;
  double* dy = a.dy + P.vm;
  wg_trsv_fwd(P.m, M, P.ldm, a.r + P.vm, a.z + P.vm, lds);
  wg_trsv_bwd(P.m, M, P.ldm, a.z + P.vm, delta, lds);
  __syncthreads();
  double dn = 0.0, yn = 0.0;
  for (int i = threadIdx.x; i < P.m; i += 256) {
    const double y2 = dy[i] + delta[i];
    dy[i] = y2;
    dn = fmax(dn, fabs(delta[i]));
    yn = fmax(yn, fabs(y2));
  }
  // max norms over the workgroup (a NaN poisons them: fmax would drop it)
  int bad = 0;
  for (int i = threadIdx.x; i < P.m; i += 256) bad |= !isfinite(delta[i]) | !isfinite(dy[i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    dn = fmax(dn, __shfl_xor(dn, o, 64));
    yn = fmax(yn, __shfl_xor(yn, o, 64));
  }
  __shared__ double s_dn[4], s_yn[4];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  if ((threadIdx.x & 63) == 0) {
    s_dn[threadIdx.x >> 6] = dn;
    s_yn[threadIdx.x >> 6] = yn;
  }
  __syncthreads();
  if (bad) atomicOr(&s_bad, 1);
  __syncthreads();
  if (threadIdx.x != 0) return;
  dn = fmax(fmax(s_dn[0], s_dn[1]), fmax(s_dn[2], s_dn[3]));
  yn = fmax(fmax(s_yn[0], s_yn[1]), fmax(s_yn[2], s_yn[3]));
  const int step = a.ref_steps[lp];
  a.ref_steps[lp] = step + 1;
  int stt = kRefRun;
  if (s_bad || !(yn > 0)) {
    stt = kRefFail;
  } else {
    const double rel = dn / yn;
    if (rel <= a.refine_tol) {
      stt = kRefOk;
    } else if (step > 0) {
      const double q = dn / a.ref_prev[lp];
      if (!(q < 0.5)) stt = kRefFail;                            // stagnation
      else if (rel * q / (1.0 - q) <= a.refine_tol) stt = kRefOk;
    }
  }
  a.ref_prev[lp] = dn;
  a.ref_status[lp] = stt;
  if (stt != kRefRun) a.refm[lp] = 0;
}

// FP32 attempts that did not converge take the FP64 factor now and from now on.
__global__ void k_bmix_end(BatchArgs a) {
  const int lp = blockIdx.x * 256 + threadIdx.x;
  if (lp >= a.count || !a.m32[lp]) return;
  a.refm[lp] = 0;
  if (a.ref_status[lp] == kRefOk) return;
  a.ref_status[lp] = kRefFail;
  a.fp32_mode[lp] = 0;
  a.go64[lp] = 1;
  a.fail[lp] = INT_MAX;
  a.minp[lp] = 0x7ff0000000000000ull;
}

}  // namespace

void launch_batch_step(hipStream_t st, const BatchArgs& a, int max_m, int k,
                       const BatchAdj* adj) {
  const int count = a.count;
  int* err = adj ? adj->err : nullptr;
  if (k < 0) hipLaunchKernelGGL(k_bclear, dim3(1), dim3(64), 0, st, a.active);
  hipLaunchKernelGGL(k_bbegin, dim3(count), dim3(256), 0, st, a, k);
  // the FP64 factor: every stepping LP, or in a mixed-precision forward
  // iteration the LPs that do not (or no longer) use the FP32 factor; the
  // normal-matrix launch forms rhs too where it covers every stepping LP
  BatchArgs a64 = a;
  int* go_main = nullptr;
  if (a.mixed && k < 0) {
    hipLaunchKernelGGL(k_brhs, dim3(cdiv(max_m, 4), count), dim3(256), 0, st, a);
    launch_bmix_factor(st, a, max_m);
    a64.go = a.go64;
    go_main = a.go;
    launch_bsyrk_normal(st, count, max_m, a.tile, a.lps, a64.go, a.A, a.d, a.M, nullptr, nullptr,
                        nullptr);
  } else if (!launch_bsyrk_normal(st, count, max_m, a.tile, a.lps, a.go, a.A, a.d, a.M, a.w, a.b,
                                  a.rhs)) {
    hipLaunchKernelGGL(k_brhs, dim3(cdiv(max_m, 4), count), dim3(256), 0, st, a);
  }
  for (int p = 0; p < max_m; p += BT) {
    launch_bpotrf_panel(st, count, max_m, a.lps, a64.go, a.M, a.diag, p, a.fail, a.minp);
    launch_bsyrk_trailing(st, count, max_m, a.tile, a.lps, a64.go, a.M, p);
  }
  launch_bdiag_to_m(st, count, max_m, a.lps, a64.go, a.M, a.diag);
  hipLaunchKernelGGL(k_btrsv, dim3(count), dim3(256), 0, st, a64, k, err, go_main);
  hipLaunchKernelGGL(k_bdir, dim3(a.nslice, count), dim3(256), 0, st, a, k);
  hipLaunchKernelGGL(k_bdir_fin, dim3(cdiv(count, 256)), dim3(256), 0, st, a, k, err);
  if (k < 0) hipLaunchKernelGGL(k_bstep, dim3(count), dim3(256), 0, st, a);
  else {
    hipLaunchKernelGGL(k_badj_t, dim3(count), dim3(256), 0, st, a, *adj, k);
    hipLaunchKernelGGL(k_badj_dyb, dim3(cdiv(max_m, 4), count), dim3(256), 0, st, a, *adj);
    hipLaunchKernelGGL(k_badj_solve, dim3(count), dim3(256), 0, st, a, *adj);
    hipLaunchKernelGGL(k_badj_h, dim3(cdiv(adj->max_n, 256), count), dim3(256), 0, st, a, *adj,
                       k);
    hipLaunchKernelGGL(k_badj_yb, dim3(cdiv(max_m, 4), count), dim3(256), 0, st, a, *adj, k);
  }
}

void launch_bmix_setup(hipStream_t st, int count, int max_m, const BatchLP* lps, const double* A,
                       float* A32) {
  hipLaunchKernelGGL(k_bmix_a32, dim3(max_m, count), dim3(256), 0, st, lps, A, A32);
}

void launch_bmix_factor(hipStream_t st, const BatchArgs& a, int max_m) {
  const int count = a.count;
  hipLaunchKernelGGL(k_bmix_begin, dim3(count), dim3(256), 0, st, a);
  launch_bsyrk_normal_f32(st, count, max_m, a.tile, a.lps, a.m32, a.A32, a.sd32, a.M32);
  for (int p = 0; p < max_m; p += BT) {
    launch_bpotrf_panel_f32(st, count, max_m, a.lps, a.m32, a.M32, a.diag32, p, a.fail, a.minp);
    launch_bsyrk_trailing_f32(st, count, max_m, a.tile, a.lps, a.m32, a.M32, p);
  }
  launch_bdiag_to_m_f32(st, count, max_m, a.lps, a.m32, a.M32, a.diag32);
  hipLaunchKernelGGL(k_bmix_solve0, dim3(count), dim3(256), 0, st, a);
  for (int q = 0; q < a.refine_max; ++q) {
    hipLaunchKernelGGL(k_bref_v, dim3(a.nslice, count), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_bref_r, dim3(cdiv(max_m, 4), count), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_bref_solve, dim3(count), dim3(256), 0, st, a);
  }
  hipLaunchKernelGGL(k_bmix_end, dim3(cdiv(count, 256)), dim3(256), 0, st, a);
}

void launch_babar(hipStream_t st, int count, int max_tiles, const BatchLP* lps,
                  const BatchState* state, const BatchAdj& adj, int tape_cap, double* Abar) {
  hipLaunchKernelGGL(k_babar, dim3(max_tiles, count), dim3(256), 0, st, lps, state, adj,
                     tape_cap, Abar);
}

void launch_batch_setup(hipStream_t st, int count, const BatchLP* lps, BatchState* state,
                        const double* Ap, const double* c, const double* x, const double* y,
                        const double* s, double* rd) {
  hipLaunchKernelGGL(k_batch_rd, dim3(count), dim3(256), 0, st, count, lps, Ap, c, y, s, rd);
  hipLaunchKernelGGL(k_batch_gap, dim3(count), dim3(256), 0, st, count, lps, state, x, s);
}

}  // namespace pdas
