// Blocked right-looking Cholesky M = L L^T of the normal matrix (Section 5.1
// names Cholesky as the usual solver for the symmetric positive definite
// A D A^T).  Row-major lower storage, panel width kTB = 64.
//
// FP64, per panel p (large matrices: panels grouped by four, see
// launch_potrf_f64):
//   1. k_chol_step: the panel step (potrf_panel_mfma: A11 and the panel rows
//      on the matrix cores, L11 to a side buffer, the rows below solved in
//      place) in its first workgroups and, in the others, the previous
//      panel's trailing update of the columns from p + 64 on (grouped: of
//      the rest of the group, and the previous group's of the rest of this
//      group beside its first panel), on tiles of the 16 x 16 x 4 FP64
//      matrix instruction;
//   2. k_chol_col0: the next panel's 64 columns updated with panel p, or
//      with the whole group when the next panel starts a new group;
//   3. grouped only, at a group's end: k_chol_upd, the group's update of the
//      columns beyond the next group, on a second stream.
// FP32 (mixed precision): potrf_panel_body, one wavefront factoring A11 with
// the panel rows solved by the other three, then the FP32 trailing update.
// Rows below the last column (mr > mc) are carried through every step like
// any other row: a right-hand side stored as row m comes out as (L^-1 r)^T,
// so the forward triangular solve costs no launch of its own.
// A pivot that is not a finite positive number is recorded (first column) in
// the iteration info and turns the step into a breakdown; no fallback.
#include <climits>
#include <cmath>
#include <utility>

#include "pdas_internal.h"
#include "syrk_tile.h"

namespace pdas {
namespace {

constexpr int NB = kTB;  // 64

template <typename T> struct RL;
template <> struct RL<double> {
  typedef double2 T2;
  __device__ static double rd(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  }
  __device__ static double rsq(double p) {
    double y = __builtin_amdgcn_rsq(p);
    double e = fma(-p * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-p * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    return y;
  }
};
template <> struct RL<float> {
  typedef float2 T2;
  __device__ static float rd(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
  }
  __device__ static float rsq(float p) {
    float y = __builtin_amdgcn_rsqf(p);
    const float e = fmaf(-p * y, y, 1.0f);
    return fmaf(0.5f * y, e, y);
  }
};

// Panel rows per workgroup: wavefronts 1..3, one row per lane.
constexpr int kRowsPerWG = 192;
constexpr int CB = 16;           // column block of the register-resident steps
constexpr int LDP = NB + 1;      // padded LDS row length

// A zero the compiler cannot see through: LDS reads indexed from it share one
// base register and carry their constant offsets as immediates.
__device__ inline int opaque_zero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}

// Marks v as live in a vector register here (emits nothing): the load that
// produced it cannot be sunk below this point into a lane-dependent branch.
__device__ inline void pin_vgpr(double& v) { asm volatile("" : "+v"(v)); }

// Workgroup wg of the panel step at column p of an mr x mc lower matrix
// (mr >= mc; rows beyond mc are extra right-hand sides stored as rows, whose
// factor rows come out as L^-1 applied to them): every workgroup factors A11
// from M; wg 0 stores L11 into diag_blk (64 x 64 row-major, lower part) and
// reports the first failing pivot column and the smallest pivot; wg >= 1 also
// solve rows p + nbe + 192 (wg - 1) ... of L21 in place.  L11 goes to the
// side block, not to M, because other workgroups of the same launch may still
// be reading A11 from M; the blocks are copied into M after the last panel.
//
// Both phases walk the 64 columns in four blocks of 16 (a runtime loop, so the
// code stays small): inside a block a lane keeps its 16 entries in registers
// and the 16 steps are unrolled (compile-time register indices); the block's
// contribution to the later columns is then applied as a rank-16 update
// through LDS.
template <typename T>
__device__ __forceinline__ void potrf_panel_body(int mr, int mc, T* __restrict__ M, long ld, int p,
                                                 int wg, T* __restrict__ diag_blk, int* fail_out,
                                                 unsigned long long* minp_bits_out) {
  __shared__ T L[NB * LDP];            // A11 on entry, L11 (row-major, lower) after phase 1
  __shared__ T col[2][CB];             // column of the current step (double-buffered)
  __shared__ T dinv[NB];               // 1 / L11[j][j]
  __shared__ T S[kRowsPerWG * LDP];    // staged panel rows of this workgroup
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nbe = min(NB, mc - p);
  const bool solve = wg > 0;
  const long r0 = (long)p + nbe + (long)(wg - 1) * kRowsPerWG;

  // stage A11 (identity beyond the matrix; upper part never read) and the
  // workgroup's panel rows, coalesced; full panels with 16-byte loads that are
  // all issued before the first LDS store
  if (nbe == NB) {
    typedef typename RL<T>::T2 T2;
    constexpr int PA = NB * NB / 2 / 256, PS = kRowsPerWG * NB / 2 / 256;
    T2 va[PA], vs[PS];
#pragma unroll
    for (int it = 0; it < PA; ++it) {
      const int e = tid + 256 * it, r = e / (NB / 2), kp = 2 * (e % (NB / 2));
      va[it] = *reinterpret_cast<const T2*>(M + (long)(p + r) * ld + p + kp);
    }
    if (solve) {
#pragma unroll
      for (int it = 0; it < PS; ++it) {
        const int e = tid + 256 * it, row = e / (NB / 2), kp = 2 * (e % (NB / 2));
        const long gr = min(r0 + row, (long)mr - 1);
        vs[it] = *reinterpret_cast<const T2*>(M + gr * ld + p + kp);
      }
    }
#pragma unroll
    for (int it = 0; it < PA; ++it) {
      const int e = tid + 256 * it, r = e / (NB / 2), kp = 2 * (e % (NB / 2));
      L[r * LDP + kp] = va[it].x;
      L[r * LDP + kp + 1] = va[it].y;
    }
    if (solve) {
#pragma unroll
      for (int it = 0; it < PS; ++it) {
        const int e = tid + 256 * it, row = e / (NB / 2), kp = 2 * (e % (NB / 2));
        S[row * LDP + kp] = vs[it].x;
        S[row * LDP + kp + 1] = vs[it].y;
      }
    }
  } else {
    // last, partial panel (its rows below are extra right-hand-side rows):
    // columns clamped to the panel, identity beyond it
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB, k = e % NB;
      const T v = M[(long)(p + min(r, nbe - 1)) * ld + p + min(k, nbe - 1)];
      L[r * LDP + k] = (r < nbe && k < nbe) ? v : ((r == k) ? T(1) : T(0));
    }
    if (solve) {
      for (int e = tid; e < kRowsPerWG * NB; e += 256) {
        const int row = e / NB, k = e % NB;
        const long gr = min(r0 + row, (long)mr - 1);
        S[row * LDP + k] = M[gr * ld + p + min(k, nbe - 1)];
      }
    }
  }
  __syncthreads();

  if (wv == 0) {
    // ---- phase 1: L11 by right-looking steps, lane i = row i ----
    const int i = lane;
    int fail = -1;
    T minp = T(INFINITY);
#pragma unroll 1
    for (int c0 = 0; c0 < NB; c0 += CB) {
      T a[CB];
#pragma unroll
      for (int jj = 0; jj < CB; ++jj) a[jj] = L[i * LDP + c0 + jj];
      T piv = RL<T>::rd(a[0], c0);
      T rinv = RL<T>::rsq(piv);
#pragma unroll
      for (int jj = 0; jj < CB; ++jj) {
        const int j = c0 + jj;
        const bool bad = !((piv > T(0)) & (piv < T(INFINITY)));
        fail = ((j < nbe) & (fail < 0) & bad) ? j : fail;
        minp = ((j < nbe) & (piv < minp)) ? piv : minp;
        const T lij = a[jj] * rinv;  // lane j: piv * rinv = L[j][j]
        a[jj] = lij;
        dinv[j] = rinv;              // same value from every lane
        if (jj + 1 < CB) {
          if (i > j && i < c0 + CB) col[jj & 1][i - c0] = lij;
          __builtin_amdgcn_wave_barrier();
          // next pivot straight from lane j+1; its reciprocal square root
          // overlaps this step's updates
          const T pn = RL<T>::rd(a[jj + 1], j + 1);
          const T l1 = RL<T>::rd(lij, j + 1);
          piv = fma(-l1, l1, pn);
          const T rnext = RL<T>::rsq(piv);
#pragma unroll
          for (int kk = jj + 1; kk < CB; ++kk) a[kk] = fma(-lij, col[jj & 1][kk], a[kk]);
          rinv = rnext;
        }
      }
#pragma unroll
      for (int jj = 0; jj < CB; ++jj) L[i * LDP + c0 + jj] = a[jj];
      __builtin_amdgcn_wave_barrier();
      // rank-16 update of the later columns, four at a time:
      // L[i][k] -= sum_jj a[jj] L[k][c0 + jj]
#pragma unroll 1
      for (int k = c0 + CB; k < NB; k += 4) {
        T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const T* lk = L + (k + u) * LDP + c0;
#pragma unroll
          for (int jj = 0; jj < CB; ++jj) acc[u] = fma(a[jj], lk[jj], acc[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) L[i * LDP + k + u] -= acc[u];
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (wg == 0 && i == 0) {
      if (fail >= 0) atomicMin(fail_out, p + fail);
      if (minp < T(INFINITY)) {
        const double mp = minp > T(0) ? (double)minp : 0.0;
        // positive doubles order like their bit patterns
        atomicMin(minp_bits_out, (unsigned long long)__double_as_longlong(mp));
      }
    }
  }
  __syncthreads();
  if (!solve) {
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB, k = e % NB;
      if (r < nbe && k <= r) diag_blk[e] = L[r * LDP + k];
    }
    return;
  }
  if (wv != 0) {
    // ---- phase 2: X L11^T = M21 by forward substitution, lane = panel row ----
    const int row = (wv - 1) * 64 + lane;
    T* xs = S + row * LDP;
#pragma unroll 1
    for (int c0 = 0; c0 < NB; c0 += CB) {
      T x[CB];
#pragma unroll
      for (int jj = 0; jj < CB; ++jj) x[jj] = xs[c0 + jj];
#pragma unroll
      for (int jj = 0; jj < CB; ++jj) {
        x[jj] *= dinv[c0 + jj];
        const T* lc = L + c0 + jj;
#pragma unroll
        for (int kk = jj + 1; kk < CB; ++kk) x[kk] = fma(-x[jj], lc[(c0 + kk) * LDP], x[kk]);
      }
#pragma unroll
      for (int jj = 0; jj < CB; ++jj) xs[c0 + jj] = x[jj];
#pragma unroll 1
      for (int k = c0 + CB; k < NB; k += 4) {
        T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const T* lk = L + (k + u) * LDP + c0;
#pragma unroll
          for (int jj = 0; jj < CB; ++jj) acc[u] = fma(x[jj], lk[jj], acc[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xs[k + u] -= acc[u];
      }
    }
  }
  __syncthreads();
  // solved rows back to M, coalesced
  for (int e = tid; e < kRowsPerWG * NB; e += 256) {
    const int row = e / NB, k = e % NB;
    if (r0 + row < mr && k < nbe) M[(r0 + row) * ld + p + k] = S[row * LDP + k];
  }
}

// ---------------------------------------------------------------------------
// FP64 panel on the matrix cores.
//
// Same step as potrf_panel_body, organised for the matrix cores.
// v_mfma_f64_4x4x4f64 computes four independent 4 x 4 x 4 products: for block
// blk, lane i + 4 blk + 16 k supplies A[i][k], lane j + 4 blk + 16 k supplies
// B[k][j] and lane j + 4 blk + 16 i receives D[i][j].  A 16 x 16 x 4 product
// C += A B is four of them: instruction cb takes rows 4 cb .. 4 cb + 3 of A
// (the same in every block) against the four column blocks of B, so lane l
// supplies B[l / 16][l % 16] and ends with C[4 cb + l / 16][l % 16] in slot
// cb.  (The single 16x16x4 FP64 instruction
// has the same result layout but runs at well under half the rate of the
// 4x4x4 one on this chip.)  Every wavefront owns rows of the panel in tiles
// of 16: wavefront 0 the 64 rows of A11 (in L), wavefronts 1..3 TPW tiles of
// staged panel rows each (in S).  The 64 columns go in four blocks of 16;
// for block b:
//   1. every wavefront forms, for each of its tiles, the block's 16 columns
//      minus the contributions of the columns already finished,
//        R = X[:, c0:c0+16] - X[:, 0:c0] L[c0:c0+16, 0:c0]^T,
//      on the matrix cores, transposed (R^T = L_blk X^T, so that R^T in the
//      result layout is directly the B operand of step 3);
//   2. wavefront 0 moves the 16 x 16 diagonal sub-block to lanes 0..15 (one
//      row per lane) and factors it column by column; lanes 16..31 carry the
//      identity rows through the same steps and so come out as the columns of
//      the inverse of the sub-block's factor;
//   3. after one barrier every wavefront multiplies its tiles below the
//      sub-block by that inverse (X_blk = R L_bb^-T, again transposed on the
//      matrix cores) and stores them; a second barrier publishes the new
//      columns for the next block.
// The row operations are those of the column-by-column factorisation and
// forward substitution, grouped in 16-column blocks; only the summation
// order differs.
typedef double mf4 __attribute__((ext_vector_type(4)));
constexpr int LDQ = NB + 4;  // padded row length: conflict-free operand reads
constexpr int YP = CB + 1;   // 16 x 16 sub-block exchange
constexpr int LIP = CB + 4;  // inverse of the sub-block's factor

// 1/sqrt(p): the hardware estimate (relative error about 2^-23) refined by
// one second-order step, y (1 + e/2 + 3e^2/8) with e = 1 - p y^2, which
// leaves an error far below an ulp before the last rounding
__device__ __forceinline__ double rsq_f64(double p) {
  const double y = __builtin_amdgcn_rsq(p);
  const double e = fma(-p * y, y, 1.0);
  const double h = fma(e, 0.375, 0.5);
  return fma(y * e, h, y);
}

template <int TPW>
struct PanelShape {
  static constexpr int rows = 3 * 16 * TPW;  // staged panel rows per workgroup
};

// C (16 x 16, slot cb = rows 4 cb + lane / 16) += A (16 x 4) B (4 x 16) with
// a[cb] = A[4 cb + lane % 4][lane / 16] and b = B[lane / 16][lane % 16]
__device__ __forceinline__ mf4 mm16(const double (&a)[4], double b, mf4 c) {
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) c[cb] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[cb], b, c[cb], 0, 0, 0);
  return c;
}

// Step 1 of a block for NTL tiles of a wavefront's rows, starting at tile
// `first` of own: R[t] = the block's columns c0 .. c0 + 15 of the tile minus
// the contributions of columns 0 .. c0 - 1, transposed (R[t][v] holds column
// lane / 16 + 4 v of row lane % 16).
template <int NTL, int NK>
__device__ __forceinline__ void panel_ustep(const double* L, const double* own, int c0, int first,
                                            int lane, mf4 (&R)[4]) {
  const int li = lane & 15, lq = lane >> 4;
  const double* rows = own + (16 * first + li) * LDQ;
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) R[t][v] = rows[16 * t * LDQ + c0 + lq + 4 * v];
  if (NK == 0) return;
  // NK = c0 / 4 K-steps, fully unrolled: every operand load can be issued
  // ahead of the matrix work that needs it
  mf4 acc[NTL];
#pragma unroll
  for (int t = 0; t < NTL; ++t) acc[t] = mf4{0.0, 0.0, 0.0, 0.0};
  const double* arow = L + (c0 + (lane & 3)) * LDQ + lq;
#pragma unroll
  for (int kq = 0; kq < NK; ++kq) {
    double a[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) a[cb] = arow[4 * cb * LDQ + 4 * kq];
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[t] = mm16(a, rows[16 * t * LDQ + 4 * kq + lq], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < NTL; ++t) R[t] -= acc[t];
}

// Step 3 of a block: tiles T0 .. NTL - 1 (from tile `first` of own) times
// the inverse of the sub-block's factor, stored as the block's columns.
template <int NTL, int T0>
__device__ __forceinline__ void panel_sstep(const double* LI, double* own, int c0, int first,
                                            int lane, const mf4 (&R)[4]) {
  const int li = lane & 15, lq = lane >> 4;
  double ai[4][4];
#pragma unroll
  for (int kq = 0; kq < 4; ++kq)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) ai[kq][cb] = LI[(4 * kq + lq) * LIP + 4 * cb + (lane & 3)];
  double* rows = own + (16 * first + li) * LDQ + c0 + lq;
#pragma unroll
  for (int t = T0; t < NTL; ++t) {
    mf4 x = mf4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) x = mm16(ai[kq], R[t][kq], x);
#pragma unroll
    for (int v = 0; v < 4; ++v) rows[16 * t * LDQ + 4 * v] = x[v];
  }
}

// LDS of the panel routine (doubles)
template <int TPW>
constexpr int panel_lds_doubles() {
  return NB * LDQ + PanelShape<TPW>::rows * LDQ + CB * YP + CB * LIP + 2 * 64 + NB + CB;
}

// wg: the workgroup's index among the panel's workgroups (workgroup 0 also
// stores the diagonal block and reports the pivots); rblk: its block of RW
// panel rows below A11, or -1 for none.
template <int TPW>
__device__ __forceinline__ void potrf_panel_mfma(int mr, int mc, double* __restrict__ M, long ld,
                                                 int p, int wg, int rblk,
                                                 double* __restrict__ diag_blk, int* fail_out,
                                                 unsigned long long* minp_bits_out, double* lds) {
  constexpr int RW = PanelShape<TPW>::rows;
  double* L = lds;                       // A11 on entry, L11 (row-major, lower) at the end
  double* S = L + NB * LDQ;              // staged panel rows of this workgroup
  double* Y = S + RW * LDQ;              // diagonal sub-block, one row per lane
  double* LI = Y + CB * YP;              // LI[q][c] = (L_bb^-1)[c][q]
  double(*CL)[64] = reinterpret_cast<double(*)[64]>(LI + CB * LIP);  // multipliers of a step
  double* PV = LI + CB * LIP + 2 * 64;   // pivots (+ CB unused), checked after the last block
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int nbe = min(NB, mc - p);
  const long r0 = (long)p + nbe + (long)rblk * RW;
  const bool solve = rblk >= 0 && r0 < mr;

  // stage A11 (identity beyond the matrix) and the workgroup's panel rows
  if (nbe == NB) {
    constexpr int PA = NB * NB / 2 / 256, PS = RW * NB / 2 / 256;
    double2 va[PA], vs[PS];
#pragma unroll
    for (int it = 0; it < PA; ++it) {
      const int e = tid + 256 * it, r = e / (NB / 2), kp = 2 * (e % (NB / 2));
      va[it] = *reinterpret_cast<const double2*>(M + (long)(p + r) * ld + p + kp);
    }
    // (a workgroup without rows stages rows too, clamped into the matrix,
    // and ignores them: unconditional staging keeps vs in registers)
#pragma unroll
    for (int it = 0; it < PS; ++it) {
      const int e = tid + 256 * it, row = e / (NB / 2), kp = 2 * (e % (NB / 2));
      const long gr = min(max(r0 + row, 0L), (long)mr - 1);
      vs[it] = *reinterpret_cast<const double2*>(M + gr * ld + p + kp);
    }
#pragma unroll
    for (int it = 0; it < PA; ++it) {
      const int e = tid + 256 * it, r = e / (NB / 2), kp = 2 * (e % (NB / 2));
      *reinterpret_cast<double2*>(L + r * LDQ + kp) = va[it];
    }
#pragma unroll
    for (int it = 0; it < PS; ++it) {
      const int e = tid + 256 * it, row = e / (NB / 2), kp = 2 * (e % (NB / 2));
      *reinterpret_cast<double2*>(S + row * LDQ + kp) = vs[it];
    }
  } else {
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB, k = e % NB;
      const double v = M[(long)(p + min(r, nbe - 1)) * ld + p + min(k, nbe - 1)];
      L[r * LDQ + k] = (r < nbe && k < nbe) ? v : ((r == k) ? 1.0 : 0.0);
    }
    if (solve) {
      for (int e = tid; e < RW * NB; e += 256) {
        const int row = e / NB, k = e % NB;
        const long gr = min(r0 + row, (long)mr - 1);
        S[row * LDQ + k] = M[gr * ld + p + min(k, nbe - 1)];
      }
    }
  }
  __syncthreads();

  // this wavefront's rows in 16-row tiles from own; wavefront 0 works on its
  // tiles from the diagonal sub-block down (tile b in block b), so its tile
  // count depends on b: each count is its own instantiation, which keeps
  // every register index and every matrix-core group free of branches
  double* own = wv == 0 ? L : S + (wv - 1) * (16 * TPW) * LDQ;
#pragma unroll 1
  for (int b = 0; b < NB / CB; ++b) {
    const int c0 = b * CB;
    mf4 R[4];
    if (wv == 0) {
      switch (b) {
        case 0: panel_ustep<4, 0>(L, own, c0, 0, lane, R); break;
        case 1: panel_ustep<3, 4>(L, own, c0, 1, lane, R); break;
        case 2: panel_ustep<2, 8>(L, own, c0, 2, lane, R); break;
        default: panel_ustep<1, 12>(L, own, c0, 3, lane, R); break;
      }
      // the sub-block (R[0]) to one row per lane, upper part zeroed; lanes
      // 16..31 start from the identity rows; lanes 32..63 repeat lanes
      // 0..31 (same rows, same steps, same values), so that every lane has
      // something to store at the end and no store needs a branch
#pragma unroll
      for (int v = 0; v < 4; ++v) Y[li * YP + lq + 4 * v] = R[0][v];
      __builtin_amdgcn_wave_barrier();
      // all 16 reads are issued by every lane before any select (pinned, so
      // the compiler cannot sink each read into a branch of its own, which
      // costs one full LDS round trip per column)
      const int lh = lane & 31;
      double y[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c) y[c] = Y[li * YP + c];
      double d = Y[li * YP + li];
#pragma unroll
      for (int c = 0; c < CB; ++c) pin_vgpr(y[c]);
      pin_vgpr(d);
      d = lh < 16 ? d : 0.0;
#pragma unroll
      for (int c = 0; c < CB; ++c)
        y[c] = lh < 16 ? (c <= lh ? y[c] : 0.0) : (lh - 16 == c ? 1.0 : 0.0);
      __builtin_amdgcn_wave_barrier();
      // step jj scales the pivot's column by the pivot's reciprocal square
      // root and takes it out of the later columns.  The pivot chain runs on
      // each lane's own diagonal entry (d, updated with its own multiplier,
      // handed over with one readlane), so only the off-diagonal updates need
      // the other rows' multipliers: they are broadcast through LDS and
      // applied one step late, filling the latency of the next pivot's
      // reciprocal square root.  No lane-dependent branch inside the steps
      // or in the stores after them (every lane stores its multiplier, lanes
      // from 16 into slots nobody reads; lane jj keeps pivot jj by a
      // select), so the 16 steps form one straight-line block the scheduler
      // can interleave.
      double piv = RL<double>::rd(d, 0);
      double rinv = rsq_f64(piv);
      // lane index re-read per block: the 16 comparisons of the pivot
      // selects stay inside the block (hoisted, their masks would not fit
      // the scalar registers)
      const int li_b = li + opaque_zero();
      double mypiv = 0.0, lprev = 0.0, clp[CB], cln[CB];
#pragma unroll
      for (int kk = 0; kk < CB; ++kk) clp[kk] = cln[kk] = 0.0;
#pragma unroll
      for (int jj = 0; jj < CB; ++jj) {
        const double lij = y[jj] * rinv;
        y[jj] = lij;
        mypiv = li_b == jj ? d : mypiv;  // lane jj's d before step jj is pivot jj
        double rnext = 0.0;
        if (jj + 1 < CB) {
          d = fma(-lij, lij, d);
          piv = RL<double>::rd(d, jj + 1);
          rnext = rsq_f64(piv);
        }
        // previous step's updates of columns jj + 1 ...
#pragma unroll
        for (int kk = jj + 1; kk < CB; ++kk)
          if (jj >= 1) y[kk] = fma(-lprev, clp[kk], y[kk]);
        if (jj + 1 < CB) {
          y[jj + 1] = fma(-lij, RL<double>::rd(lij, jj + 1), y[jj + 1]);
          CL[jj & 1][lane] = lij;
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int kk = jj + 2; kk < CB; ++kk) cln[kk] = CL[jj & 1][kk];
        }
        lprev = lij;
#pragma unroll
        for (int kk = 0; kk < CB; ++kk) clp[kk] = cln[kk];
        rinv = rnext;
      }
      // rows of L11 (lanes 0..15) and columns of the inverse (lanes 16..31,
      // stored as rows of LI), 16 consecutive doubles per lane; pivots of
      // lanes 16..31 go to unused slots
      double* dst = lh < 16 ? L + (c0 + li) * LDQ + c0 : LI + li * LIP;
#pragma unroll
      for (int c = 0; c < CB; ++c) dst[c] = y[c];
      PV[(lh < 16 ? c0 : NB) + li] = mypiv;
    } else if (solve) {
      switch (b) {
        case 0: panel_ustep<TPW, 0>(L, own, c0, 0, lane, R); break;
        case 1: panel_ustep<TPW, 4>(L, own, c0, 0, lane, R); break;
        case 2: panel_ustep<TPW, 8>(L, own, c0, 0, lane, R); break;
        default: panel_ustep<TPW, 12>(L, own, c0, 0, lane, R); break;
      }
    }
    __syncthreads();
    if (wv == 0) {
      switch (b) {
        case 0: panel_sstep<4, 1>(LI, own, c0, 0, lane, R); break;
        case 1: panel_sstep<3, 1>(LI, own, c0, 1, lane, R); break;
        case 2: panel_sstep<2, 1>(LI, own, c0, 2, lane, R); break;
        default: break;
      }
    } else if (solve) {
      panel_sstep<TPW, 0>(LI, own, c0, 0, lane, R);
    }
    __syncthreads();
    // the block's 16 finished columns of the panel rows go out now, written
    // by wavefronts 1..3 only: wavefront 0 goes straight on to the next
    // block's sub-block and factor chain, the critical path, while the
    // others have slack until the next barrier (after the last block all
    // four share the stores)
    const bool last = b == NB / CB - 1;
    if (solve && (wv > 0 || last)) {
      const int t0 = last ? tid : tid - 64, nt = last ? 256 : 192;
      for (int e = t0; e < RW * CB; e += nt) {
        const int row = e / CB, k = c0 + e % CB;
        if (r0 + row < mr && k < nbe) M[(r0 + row) * ld + p + k] = S[row * LDQ + k];
      }
    }
  }

  if (wv == 0 && wg == 0) {
    // first failing pivot column and smallest pivot (lane j: column j)
    const double pv = PV[lane];
    const bool inb = lane < nbe;
    int fail = (inb && !((pv > 0.0) & (pv < INFINITY))) ? lane : INT_MAX;
    double minp = (inb && pv < INFINITY) ? pv : INFINITY;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      fail = min(fail, __shfl_xor(fail, o, 64));
      const double mo = __shfl_xor(minp, o, 64);
      minp = mo < minp ? mo : minp;
    }
    if (lane == 0) {
      if (fail != INT_MAX) atomicMin(fail_out, p + fail);
      if (minp < INFINITY) {
        const double mp = minp > 0.0 ? minp : 0.0;
        // positive doubles order like their bit patterns
        atomicMin(minp_bits_out, (unsigned long long)__double_as_longlong(mp));
      }
    }
  }
  if (wg == 0) {
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB, k = e % NB;
      if (r < nbe && k <= r) diag_blk[e] = L[r * LDQ + k];
    }
  }
}

// FP64 panel rows per workgroup (16-row tiles per wavefront 1..3)
constexpr int kPanelTPW = 1;
constexpr int kPanelRows = PanelShape<kPanelTPW>::rows;

// ---------------------------------------------------------------------------
// Trailing updates:
//   C[i][j] -= sum_{k < K} X[i][k] X[j][k]
// over a lower trapezoid: rows [0, mm) and columns [0, ncols) of C (j <= i),
// with X the factor's rows at the same offsets (K = 64 for one panel, 64 G
// for a group of G panels).  One BM x BM tile per workgroup on the
// 16 x 16 x 4 FP64 matrix instruction (lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; slot v of the result is D[l / 16 + 4 v][l % 16]):
// 2 x 2 wavefronts of BM/2 x BM/2 (blocks of 16 x 16), operands
// through double-buffered LDS in stages of 16 along K with rows padded to 18
// doubles.  The accumulators start from the C values (loaded beside the
// first stage, so their latency overlaps it) and the row operand is staged
// negated, so the matrix instructions leave C - X X^T directly.
// BM = 128 for the grouped schedule's large update on the second stream
// (fewer, longer tiles: each operand row is reused by twice the columns);
// BM = 64 beside a panel, where the update must finish within the step.
constexpr int kUpKC = 16, kUpLS = kUpKC + 2;
template <int BM>
constexpr int up_lds_doubles() {
  return 2 * 2 * BM * kUpLS;
}

struct CholUpd {
  int c0;      // C and the row operand start at row and column c0 of M
  int ncols;   // columns c0 .. c0 + ncols - 1 are updated
  int kcol;    // factor columns kcol .. kcol + K - 1 are applied
  int K;       // a multiple of 32
  int nrt;     // row tiles: cdiv(mr - c0, BM)
  int ntiles;  // tiles of the trapezoid
};

__host__ __device__ inline int trap_tiles(int nrt, int nct) {
  return nct * nrt - nct * (nct - 1) / 2;
}

// Tile t of the trapezoid, column by column: column tj holds row tiles
// tj .. nrt - 1.
__device__ inline void trap_coords(int t, int nrt, int& ti, int& tj) {
  tj = 0;
  while (t >= nrt - tj) {
    t -= nrt - tj;
    ++tj;
  }
  ti = tj + t;
}

// NT threads: 256 (2 x 2 wavefronts of BM/2 x BM/2) or 512 (2 x 4
// wavefronts of BM/2 x BM/4, two per SIMD, for a launch with one workgroup
// per compute unit); the per-element arithmetic is the same either way.
template <int BM, int NT = 256>
__device__ __forceinline__ void chol_update_tile(int mr, const CholUpd& u, double* __restrict__ M,
                                                 long ld, int t, double* __restrict__ lds) {
  typedef double upd4 __attribute__((ext_vector_type(4)));
  static_assert(NT == 256 || NT == 512, "2 x 2 or 2 x 4 wavefronts");
  constexpr int PPR = kUpKC / 2;              // element pairs per row per stage
  constexpr int PAIRS = BM * PPR / NT;        // pairs per thread per operand
  constexpr int WCS = NT / 128;               // wavefront columns
  constexpr int WR = BM / 2, WC = BM / WCS;   // wavefront block rows and columns
  constexpr int NBR = WR / 16, NBC = WC / 16; // 16 x 16 blocks per wavefront
  int ti, tj;
  trap_coords(t, u.nrt, ti, tj);
  const int mm = mr - u.c0;
  const int row0 = ti * BM, col0 = tj * BM;
  const double* X = M + (long)u.c0 * ld + u.kcol;
  double* C = M + (long)u.c0 * ld + u.c0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr0 = (wv / WCS) * WR, wc0 = (wv % WCS) * WC;
  // a wavefront whose block lies above the diagonal of a diagonal tile idles
  const bool active = !(ti == tj && wr0 + WR <= wc0);
  upd4 acc[NBR][NBC];
#pragma unroll
  for (int r = 0; r < NBR; ++r)
#pragma unroll
    for (int c = 0; c < NBC; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = min(row0 + wr0 + 16 * r + lk + 4 * v, mm - 1);
        const int gc = min(col0 + wc0 + 16 * c + li, gr);
        acc[r][c][v] = active ? C[(long)gr * ld + gc] : 0.0;
      }
  double(*buf)[2][BM * kUpLS] = reinterpret_cast<double(*)[2][BM * kUpLS]>(lds);
  double2 pa[PAIRS], pb[PAIRS];
  // every load address is clamped into the matrix; rows outside the tile
  // are zeroed when staged (K is a multiple of the stage length)
  auto gload = [&](int st) {
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int q = tid + NT * it;
      const int row = q / PPR, k = st * kUpKC + 2 * (q % PPR);
      const long ra = min(row0 + row, mm - 1), rb = min(col0 + row, mm - 1);
      pa[it] = *reinterpret_cast<const double2*>(X + ra * ld + k);
      pb[it] = *reinterpret_cast<const double2*>(X + rb * ld + k);
    }
  };
  auto sstore = [&](int b) {
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int q = tid + NT * it;
      const int row = q / PPR, kk = 2 * (q % PPR);
      // element-wise selects (a select of whole vectors went through memory)
      const bool va = row0 + row < mm, vb = col0 + row < mm;
      double2 sa, sb;
      sa.x = va ? -pa[it].x : 0.0;
      sa.y = va ? -pa[it].y : 0.0;
      sb.x = vb ? pb[it].x : 0.0;
      sb.y = vb ? pb[it].y : 0.0;
      *reinterpret_cast<double2*>(&buf[b][0][row * kUpLS + kk]) = sa;
      *reinterpret_cast<double2*>(&buf[b][1][row * kUpLS + kk]) = sb;
    }
  };
  const int nst = u.K / kUpKC;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) gload(st + 1);
    if (active) {
      const double* la = buf[cur][0];
      const double* lb = buf[cur][1];
#pragma unroll
      for (int ks = 0; ks < kUpKC / 4; ++ks) {
        double a[NBR], b[NBC];
#pragma unroll
        for (int r = 0; r < NBR; ++r) a[r] = la[(wr0 + 16 * r + li) * kUpLS + 4 * ks + lk];
#pragma unroll
        for (int c = 0; c < NBC; ++c) b[c] = lb[(wc0 + 16 * c + li) * kUpLS + 4 * ks + lk];
#pragma unroll
        for (int r = 0; r < NBR; ++r)
#pragma unroll
          for (int c = 0; c < NBC; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], b[c], acc[r][c], 0, 0, 0);
      }
    }
    if (st + 1 < nst) sstore(cur ^ 1);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int r = 0; r < NBR; ++r)
#pragma unroll
    for (int c = 0; c < NBC; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = row0 + wr0 + 16 * r + lk + 4 * v, gc = col0 + wc0 + 16 * c + li;
        if (gr < mm && gc <= gr && gc < u.ncols) C[(long)gr * ld + gc] = acc[r][c][v];
      }
}

// The fused Cholesky step at column p.  Workgroups 0 .. npw_need - 1 run the
// panel step; workgroups from npw (a multiple of 8, so that the tile order
// stays XCD-aware) run the tiles of up to two trailing updates (u1, then
// u2) that the grouped schedule places beside this panel.  The panel writes
// columns p .. p + 63; the updates write columns from p + 64 on and read
// only finished factor columns, so nothing in one launch races.
template <int BM>
constexpr int step_lds_doubles() {
  return panel_lds_doubles<kPanelTPW>() > up_lds_doubles<BM>() ? panel_lds_doubles<kPanelTPW>()
                                                               : up_lds_doubles<BM>();
}

template <int BM>
__global__ __launch_bounds__(256) void k_chol_step(int mr, int mc, double* __restrict__ M, long ld,
                                                   int p, double* __restrict__ diag,
                                                   DevInfo* info, int npw_need, int npw,
                                                   CholUpd u1, CholUpd u2, int per_xcd) {
  __shared__ __attribute__((aligned(16))) double lds[step_lds_doubles<BM>()];
  const int b = blockIdx.x;
  if (b < npw) {
    if (b >= npw_need) return;
    potrf_panel_mfma<kPanelTPW>(mr, mc, M, ld, p, b, b - 1, diag + (long)(p / NB) * NB * NB,
                                &info->chol_fail,
                                reinterpret_cast<unsigned long long*>(&info->min_pivot), lds);
    return;
  }
  const int bb = b - npw;
  const int t = (bb & 7) * per_xcd + (bb >> 3);
  if (t < u1.ntiles) chol_update_tile<BM>(mr, u1, M, ld, t, lds);
  else if (t - u1.ntiles < u2.ntiles) chol_update_tile<BM>(mr, u2, M, ld, t - u1.ntiles, lds);
}

// Update of the next panel's columns q .. q + NB - 1 (all rows from q) with
// the factor columns kcol .. kcol + K - 1 (K = 64: the panel just factored;
// K = 256: the group of four just finished).  This update sits on the
// critical path between two panels, so it is cut fine and kept short: 32 x
// 32 tiles (workgroup b takes tile (0, 0) for b = 0, else ((b + 1) / 2,
// (b + 1) % 2)), each wavefront a 16 x 16 block on the 16 x 16 x 4 FP64
// instruction with its operands loaded straight into registers (no LDS, no
// barrier), 64 factor columns per round with every load of the round
// issued at once; the accumulators start from C and the row operand is
// negated, so the result is C - L_r L_c^T.
constexpr int kCol0BM = 32;
__global__ __launch_bounds__(256) void k_chol_col0(int mr, double* __restrict__ M, long ld, int q,
                                                   int kcol, int K) {
  const int b = blockIdx.x;
  const int ti = (b + 1) / 2, tj = b == 0 ? 0 : (b + 1) % 2;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = q + kCol0BM * ti + 16 * (wv >> 1);  // the wavefront's block rows
  const int c0 = q + kCol0BM * tj + 16 * (wv & 1);   // and columns
  if (c0 > r0 + 15 || r0 >= mr) return;              // above the diagonal, or below the matrix
  const double* pa = M + (long)min(r0 + li, mr - 1) * ld + kcol + lk;
  const double* pb = M + (long)min(c0 + li, mr - 1) * ld + kcol + lk;
  mf4 acc;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gr = min(r0 + lk + 4 * v, mr - 1), gc = min(c0 + li, gr);
    acc[v] = M[(long)gr * ld + gc];
  }
  for (int k0 = 0; k0 < K; k0 += 64) {
    double a[16], bb[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      a[s] = -pa[k0 + 4 * s];
      bb[s] = pb[k0 + 4 * s];
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bb[s], acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gr = r0 + lk + 4 * v, gc = c0 + li;
    if (gr < mr && gc <= gr) M[(long)gr * ld + gc] = acc[v];
  }
}

// A trailing update on its own (the grouped schedule's update of the columns
// beyond the next group, on the second stream): at most one workgroup per
// compute unit, each taking every gridDim.x-th tile, so that the panels and
// column updates of the other stream always find room beside it; eight
// wavefronts per workgroup, so that each SIMD still has two (151 registers
// each: a 64-edge fused step's wavefront, 158, fits beside them).
template <int BM>
__global__ __launch_bounds__(512) void k_chol_upd(
    int mr, double* __restrict__ M, long ld, CholUpd u) {
  __shared__ __attribute__((aligned(16))) double lds[up_lds_doubles<BM>()];
  for (int t = blockIdx.x; t < u.ntiles; t += gridDim.x) {
    chol_update_tile<BM, 512>(mr, u, M, ld, t, lds);
    __syncthreads();  // the next tile restages the LDS buffers
  }
}
constexpr int kUpdGroups = 256;

__global__ __launch_bounds__(256) void k_potrf_panel_f32(int mr, int mc, float* __restrict__ M,
                                                          long ld, int p, float* __restrict__ diag,
                                                          DevInfo* info) {
  potrf_panel_body<float>(mr, mc, M, ld, p, blockIdx.x, diag + (long)(p / NB) * NB * NB,
                          &info->chol_fail,
                          reinterpret_cast<unsigned long long*>(&info->min_pivot));
}

// Diagonal blocks from the side buffer into M (lower parts); one workgroup
// per block.
template <typename T>
__device__ __forceinline__ void diag_to_m(int m, T* __restrict__ M, long ld,
                                          const T* __restrict__ diag, int q) {
  const int p = q * NB, nbe = min(NB, m - p);
  const T* blk = diag + (long)q * NB * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e / NB, k = e % NB;
    if (r < nbe && k <= r) M[(long)(p + r) * ld + p + k] = blk[e];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_diag_to_m(int m, T* __restrict__ M, long ld,
                                                    const T* __restrict__ diag) {
  diag_to_m<T>(m, M, ld, diag, blockIdx.x);
}

// Batched panel step at column p: LP = blockIdx.y (skipped unless it takes a
// step this iteration and has a panel at p).  One tile of 16 rows per
// wavefront: the smaller LDS footprint lets two workgroups share a compute
// unit, which suits the many short panels of a batch.  Workgroup x takes
// rows block x - shift below A11: shift 0 gives workgroup 0 rows as well
// (fewer workgroups), shift 1 leaves it the diagonal block alone.
constexpr int kBPanelTPW = 1;
constexpr int kBPanelRows = PanelShape<kBPanelTPW>::rows;
__global__ __launch_bounds__(256) void k_bpotrf_panel(const BatchLP* __restrict__ lps,
                                                       const int* __restrict__ go, double* Mpool,
                                                       double* diagpool, int p, int shift,
                                                       int* fail,
                                                       unsigned long long* minp_bits) {
  const int lp = blockIdx.y;
  const BatchLP P = lps[lp];
  if (!go[lp] || p >= P.m) return;
  const int below = P.m - p - min(NB, P.m - p);
  const int rblk = (int)blockIdx.x - shift;
  if (blockIdx.x > 0 && rblk * kBPanelRows >= below) return;
  __shared__ __attribute__((aligned(16))) double lds[panel_lds_doubles<kBPanelTPW>()];
  potrf_panel_mfma<kBPanelTPW>(P.m, P.m, Mpool + P.M_off, P.ldm, p, blockIdx.x, rblk,
                              diagpool + P.diag_off + (long)(p / NB) * NB * NB, fail + lp,
                              minp_bits + lp, lds);
}

// Batched FP32 panel step at column p (mixed precision): the single-LP FP32
// panel routine on M32_i for the LPs whose flag is set.
__global__ __launch_bounds__(256) void k_bpotrf_panel_f32(const BatchLP* __restrict__ lps,
                                                           const int* __restrict__ go,
                                                           float* M32, float* diag32, int p,
                                                           int* fail,
                                                           unsigned long long* minp_bits) {
  const int lp = blockIdx.y;
  const BatchLP P = lps[lp];
  if (!go[lp] || p >= P.m) return;
  const int below = P.m - p - min(NB, P.m - p);
  if ((int)blockIdx.x > (below + kRowsPerWG - 1) / kRowsPerWG) return;
  potrf_panel_body<float>(P.m, P.m, M32 + P.m32_off, P.ld32, p, blockIdx.x,
                          diag32 + P.diag_off + (long)(p / NB) * NB * NB, fail + lp,
                          minp_bits + lp);
}

__global__ __launch_bounds__(256) void k_bdiag_to_m_f32(const BatchLP* __restrict__ lps,
                                                         const int* __restrict__ go, float* M32,
                                                         const float* diag32) {
  const int lp = blockIdx.y;
  if (!go[lp]) return;
  const BatchLP P = lps[lp];
  if ((int)blockIdx.x * NB >= P.m) return;
  diag_to_m<float>(P.m, M32 + P.m32_off, P.ld32, diag32 + P.diag_off, blockIdx.x);
}

// Batched diagonal blocks into M: LP = blockIdx.y, block blockIdx.x.
__global__ __launch_bounds__(256) void k_bdiag_to_m(const BatchLP* __restrict__ lps,
                                                     const int* __restrict__ go, double* Mpool,
                                                     const double* diagpool) {
  const int lp = blockIdx.y;
  const BatchLP P = lps[lp];
  if (!go[lp] || (int)blockIdx.x * NB >= P.m) return;
  diag_to_m<double>(P.m, Mpool + P.M_off, P.ldm, diagpool + P.diag_off, blockIdx.x);
}

}  // namespace

// Right-looking schedule over panels of NB = 64 columns, optionally grouped
// by G panels.  With G = 1 every step applies the previous panel to all
// later columns (K = 64), beside the next panel.  With G > 1 a panel's
// update of the columns inside its own group is applied at once (K = 64);
// its update of the columns beyond the group is deferred and applied with
// the rest of the group as one K = 64 G update, so the trailing matrix is
// read and written once per group instead of once per panel.  For panel
// k = G g + j at column p (group columns gs .. ge):
//   step launch k: the panel, and beside it panel k - 1 on [p + 64, ge)
//     when j >= 1 (K = 64);
//     and group g - 1 (K = 64 G) on [p + 64, ge) when j = 0 and g >= 1;
//   then a column update of the next panel's 64 columns: panel k inside the
//   group, group g (K = 64 G) after the group's last panel, when group g's
//   update of the columns beyond the next group, [ne, mc), also starts on
//   the second stream, beside the next group's panels (a K = 256 tile takes
//   about as long as three panel steps, so a schedule that put those tiles
//   into the steps made every step wait for one).
// Every update reads finished factor columns only, no two concurrent
// launches write the same columns, and each element receives the updates in
// the same order and with the same instruction sequence whichever stream
// and tile routine apply them; each panel's columns have received every
// earlier panel's contribution when its step starts.
namespace {
int chol_group_min_m = 4096;
CholUpd make_upd(int bm, int mr, int c0, int c1, int kcol, int K) {
  CholUpd u{};
  u.c0 = c0;
  u.ncols = c1 - c0;
  u.kcol = kcol;
  u.K = K;
  u.nrt = mr > c0 ? cdiv(mr - c0, bm) : 0;
  u.ntiles = (u.ncols > 0 && u.nrt > 0) ? trap_tiles(u.nrt, cdiv(u.ncols, bm)) : 0;
  return u;
}
}  // namespace

bool chol_grouped(int mc) { return mc >= chol_group_min_m; }
void set_chol_group_min_m(int m) { chol_group_min_m = m; }

void launch_potrf_f64(hipStream_t st, int mr, int mc, double* M, long ld, DevInfo* info,
                      double* diag, const CholAux* aux) {
  // grouping pays where the trailing update is bound by its traffic (large
  // m); below that the per-panel update hides behind the panel itself
  const bool big = chol_grouped(mc);
  const int G = big ? 4 : 1, GW = G * NB;
  bool two = big && aux && aux->st && aux->ev_main && aux->ev_aux;
  hipStream_t sb = two ? aux->st : st;
  bool aux_pending = false;  // an update on the second stream not yet waited for
  // should an event call fail, the second stream is drained from the host
  // and the rest of the factorization runs in order on st
  auto drop_aux = [&]() {
    (void)hipStreamSynchronize(sb);
    two = false;
    sb = st;
    aux_pending = false;
  };
  for (int p = 0; p < mc; p += NB) {
    const int k = p / NB, g = k / G, j = k % G;
    const int gs = g * GW, ge = gs + GW < mc ? gs + GW : mc;
    const int nbe = (mc - p) < NB ? (mc - p) : NB;
    const int npw_need = 1 + cdiv(mr - p - nbe, kPanelRows);
    // the updates beside a panel are on the critical path (grouped: the
    // previous group's K = 256 update of the rest of the group beside its
    // first panel), so they take 64-edge tiles, a quarter of the work each;
    // their registers also leave room beside the second stream's update
    const CholUpd none = make_upd(64, mr, 0, 0, 0, NB);
    CholUpd u1 = none, u2 = none;
    if (j >= 1) u1 = make_upd(64, mr, p + NB, ge, p - NB, NB);
    // G = 1: the previous panel on all later columns; grouped: the previous
    // group on the rest of this group's columns, beside its first panel
    if (g >= 1 && (G == 1 || j == 0)) u2 = make_upd(64, mr, p + NB, G == 1 ? mc : ge, gs - GW, GW);
    const int ntiles = u1.ntiles + u2.ntiles;
    const int per_xcd = cdiv(ntiles, 8);
    const int npw = ntiles ? cdiv(npw_need, 8) * 8 : npw_need;
    hipLaunchKernelGGL(k_chol_step<64>, dim3(npw + 8 * per_xcd), dim3(256), 0, st, mr, mc, M, ld,
                       p, diag, info, npw_need, npw, u1, u2, per_xcd);
    const int q = p + NB;
    if (q >= mc) continue;
    if (!big || q < ge) {
      // the next panel's 64 columns with this panel
      hipLaunchKernelGGL(k_chol_col0, dim3(2 * cdiv(mr - q, kCol0BM) - 1), dim3(256), 0, st, mr,
                         M, ld, q, p, NB);
      continue;
    }
    // Group g is finished (its factor columns are final).  Its update of the
    // columns beyond the next group goes to the second stream, beside the
    // next group's panels, which write only their own columns; the next
    // group's first panel gets it from the column update and the rest of
    // that group from the first step, both after the previous group's update
    // of them (on the second stream) has ended.
    const int ne = ge + GW < mc ? ge + GW : mc;
    if (two && (hipEventRecord(aux->ev_main, st) != hipSuccess ||
                hipStreamWaitEvent(sb, aux->ev_main, 0) != hipSuccess))
      drop_aux();
    if (ne < mc) {
      const CholUpd uo = make_upd(128, mr, ne, mc, gs, GW);
      const int gx = uo.ntiles < kUpdGroups ? uo.ntiles : kUpdGroups;
      hipLaunchKernelGGL(k_chol_upd<128>, dim3(gx), dim3(512), 0, sb, mr, M, ld, uo);
    }
    if (two && aux_pending && hipStreamWaitEvent(st, aux->ev_aux, 0) != hipSuccess) drop_aux();
    if (two) {
      if (hipEventRecord(aux->ev_aux, sb) != hipSuccess)
        drop_aux();
      else
        aux_pending = ne < mc;
    }
    hipLaunchKernelGGL(k_chol_col0, dim3(2 * cdiv(mr - q, kCol0BM) - 1), dim3(256), 0, st, mr, M,
                       ld, q, gs, GW);
  }
  if (two && aux_pending && hipStreamWaitEvent(st, aux->ev_aux, 0) != hipSuccess) drop_aux();
  hipLaunchKernelGGL(k_diag_to_m<double>, dim3(cdiv(mc, NB)), dim3(256), 0, st, mc, M, ld, diag);
}

void launch_potrf_f32(hipStream_t st, int m, float* M, long ld, DevInfo* info, float* diag) {
  for (int p = 0; p < m; p += NB) {
    const int nbe = (m - p) < NB ? (m - p) : NB;
    const int below = m - p - nbe;
    const int grid = 1 + cdiv(below, kRowsPerWG);
    hipLaunchKernelGGL(k_potrf_panel_f32, dim3(grid), dim3(256), 0, st, m, m, M, ld, p, diag,
                       info);
    if (below > 0)
      launch_syrk_f32(st, below, NB, M + (long)(p + NB) * ld + p, ld, nullptr,
                      M + (long)(p + NB) * ld + (p + NB), ld, true, 1, nullptr);
  }
  hipLaunchKernelGGL(k_diag_to_m<float>, dim3(cdiv(m, NB)), dim3(256), 0, st, m, M, ld, diag);
}

void launch_bpotrf_panel(hipStream_t st, int count, int max_m, const BatchLP* lps, const int* go,
                         double* Mpool, double* diagpool, int p, int* fail,
                         unsigned long long* minp_bits) {
  const int below = max_m - p - NB;
  // first panel (every LP has one, most workgroups): workgroup 0 keeps to
  // the diagonal block; later panels: fewer workgroups.  Measured on a
  // ragged batch of 512 LPs with m up to 256: 67 / 41 us for the first two
  // panels against 81 / 41 (all shift 0) and 67 / 65 (all shift 1).
  const int shift = p == 0 ? 1 : 0;
  const int gx = below > 0 ? shift + cdiv(below, kBPanelRows) : 1;
  hipLaunchKernelGGL(k_bpotrf_panel, dim3(gx, count), dim3(256), 0, st, lps, go, Mpool, diagpool,
                     p, shift, fail, minp_bits);
}

void launch_bdiag_to_m(hipStream_t st, int count, int max_m, const BatchLP* lps, const int* go,
                       double* Mpool, const double* diagpool) {
  hipLaunchKernelGGL(k_bdiag_to_m, dim3(cdiv(max_m, NB), count), dim3(256), 0, st, lps, go, Mpool,
                     diagpool);
}

void launch_bpotrf_panel_f32(hipStream_t st, int count, int max_m, const BatchLP* lps,
                             const int* go, float* M32, float* diag32, int p, int* fail,
                             unsigned long long* minp_bits) {
  const int below = max_m - p - NB;
  const int gx = 1 + (below > 0 ? cdiv(below, kRowsPerWG) : 0);
  hipLaunchKernelGGL(k_bpotrf_panel_f32, dim3(gx, count), dim3(256), 0, st, lps, go, M32, diag32,
                     p, fail, minp_bits);
}

void launch_bdiag_to_m_f32(hipStream_t st, int count, int max_m, const BatchLP* lps,
                           const int* go, float* M32, const float* diag32) {
  hipLaunchKernelGGL(k_bdiag_to_m_f32, dim3(cdiv(max_m, NB), count), dim3(256), 0, st, lps, go,
                     M32, diag32);
}

}  // namespace pdas
