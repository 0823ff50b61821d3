// Blocked right-looking Cholesky M = L L^T of the normal matrix (Section 5.1
// names Cholesky as the usual solver for the symmetric positive definite
// A D A^T).  Row-major lower storage, panel width kTB = 64.
//
// Per panel p:
//   1. k_potrf_panel: wavefront 0 of every workgroup factors the 64 x 64
//      diagonal block (identical arithmetic in each, so identical results),
//      one row per lane with the whole row in registers.  Step j broadcasts
//      column j through LDS; the next pivot is taken straight from lane j+1
//      with two readlanes, so its reciprocal square root overlaps the step's
//      updates.  Every step is a template instance, so all register indices
//      are compile-time constants.  Meanwhile wavefronts 1..3 stage 192 panel
//      rows in LDS; after one barrier each of their lanes solves one row of
//      L21 = M21 L11^-T by forward substitution.  Workgroup 0 stores L11.
//   2. trailing update M22 -= L21 L21^T on the matrix cores (the normal-matrix
//      kernel in subtract mode, lower tiles only).
// Rows below the last column (mr > mc) are carried through both steps like
// any other row: a right-hand side stored as row m comes out as (L^-1 r)^T,
// so the forward triangular solve costs no launch of its own.
// The pivot reciprocal square root is the hardware estimate refined by Newton
// steps (within an ulp or two of the correctly rounded value).  A pivot that
// is not a finite positive number is recorded (first column) in the
// iteration info and turns the step into a breakdown; no fallback.
#include <climits>
#include <cmath>
#include <utility>

#include "pdas_internal.h"

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

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_panel(int mr, int mc, T* __restrict__ M, long ld,
                                                      int p, T* __restrict__ diag,
                                                      DevInfo* info) {
  potrf_panel_body<T>(mr, mc, M, ld, p, blockIdx.x, diag + (long)(p / NB) * NB * NB,
                      &info->chol_fail, reinterpret_cast<unsigned long long*>(&info->min_pivot));
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
// step this iteration and has a panel at p).
__global__ __launch_bounds__(256) void k_bpotrf_panel(const BatchLP* __restrict__ lps,
                                                       const int* __restrict__ go, double* Mpool,
                                                       double* diagpool, int p, int* fail,
                                                       unsigned long long* minp_bits) {
  const int lp = blockIdx.y;
  const BatchLP P = lps[lp];
  if (!go[lp] || p >= P.m) return;
  const int below = P.m - p - min(NB, P.m - p);
  if ((int)blockIdx.x > (below + kRowsPerWG - 1) / kRowsPerWG) return;
  potrf_panel_body<double>(P.m, P.m, Mpool + P.M_off, P.ldm, p, blockIdx.x,
                           diagpool + P.diag_off + (long)(p / NB) * NB * NB, fail + lp,
                           minp_bits + lp);
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

void launch_potrf_f64(hipStream_t st, int mr, int mc, double* M, long ld, DevInfo* info,
                      double* diag) {
  for (int p = 0; p < mc; p += NB) {
    const int nbe = (mc - p) < NB ? (mc - p) : NB;
    const int grid = 1 + cdiv(mr - p - nbe, kRowsPerWG);
    hipLaunchKernelGGL(k_potrf_panel<double>, dim3(grid), dim3(256), 0, st, mr, mc, M, ld, p,
                       diag, info);
    if (p + NB < mc) {
      launch_syrk_f64(st, mr - p - NB, NB, M + (long)(p + NB) * ld + p, ld, nullptr,
                      M + (long)(p + NB) * ld + (p + NB), ld, true, 64, 1, nullptr);
    }
  }
  hipLaunchKernelGGL(k_diag_to_m<double>, dim3(cdiv(mc, NB)), dim3(256), 0, st, mc, M, ld, diag);
}

void launch_potrf_f32(hipStream_t st, int m, float* M, long ld, DevInfo* info, float* diag) {
  for (int p = 0; p < m; p += NB) {
    const int nbe = (m - p) < NB ? (m - p) : NB;
    const int below = m - p - nbe;
    const int grid = 1 + cdiv(below, kRowsPerWG);
    hipLaunchKernelGGL(k_potrf_panel<float>, dim3(grid), dim3(256), 0, st, m, m, M, ld, p, diag,
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
  const int gx = 1 + (below > 0 ? cdiv(below, kRowsPerWG) : 0);
  hipLaunchKernelGGL(k_bpotrf_panel, dim3(gx, count), dim3(256), 0, st, lps, go, Mpool, diagpool,
                     p, fail, minp_bits);
}

void launch_bdiag_to_m(hipStream_t st, int count, int max_m, const BatchLP* lps, const int* go,
                       double* Mpool, const double* diagpool) {
  hipLaunchKernelGGL(k_bdiag_to_m, dim3(cdiv(max_m, NB), count), dim3(256), 0, st, lps, go, Mpool,
                     diagpool);
}

}  // namespace pdas
