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

// A zero the compiler cannot see through: LDS reads indexed from it share one
// base register and carry their constant offsets as immediates.
__device__ inline int opaque_zero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}


template <typename T>
struct FactorState {
  T piv, rinv, myrinv, minp;
  int fail;
};

// One right-looking step j of the unblocked factorization of the diagonal
// block held one row per lane (a[k] = entry (lane, k)); j is a template
// parameter so every register index is a compile-time constant.
template <typename T, int J>
__device__ __forceinline__ void factor_step(T (&a)[NB], FactorState<T>& fs, int nbe, int i,
                                            T (*col)[NB], int z0) {
  const bool valid = J < nbe;
  const T piv = fs.piv, rinv = fs.rinv;
  const bool bad = !((piv > T(0)) & (piv < T(INFINITY)));
  fs.fail = (valid & (fs.fail < 0) & bad) ? J : fs.fail;
  fs.minp = (valid & (piv < fs.minp)) ? piv : fs.minp;
  const T lij = a[J] * rinv;  // lane J: piv * rinv = L[J][J]
  a[J] = lij;
  fs.myrinv = (i == J) ? rinv : fs.myrinv;
  if constexpr (J + 1 < NB) {
    col[J & 1][i] = lij;
    __builtin_amdgcn_wave_barrier();
    // next pivot straight from lane J+1, off the LDS path; its reciprocal
    // square root overlaps this step's updates
    const T pn = RL<T>::rd(a[J + 1], J + 1);
    const T l1 = RL<T>::rd(lij, J + 1);
    fs.piv = fma(-l1, l1, pn);
    const T rnext = RL<T>::rsq(fs.piv);
    const T* cj = col[J & 1] + z0;
    // column values in chunks, the next chunk's reads issued ahead of the
    // current chunk's updates
    constexpr int CH = 16, K0 = J + 1, NCH = (NB - K0 + CH - 1) / CH;
    T cv[NCH][CH];
#pragma unroll
    for (int kk = 0; kk < CH; ++kk)
      if (K0 + kk < NB) cv[0][kk] = cj[K0 + kk];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      if (c + 1 < NCH) {
#pragma unroll
        for (int kk = 0; kk < CH; ++kk)
          if (K0 + (c + 1) * CH + kk < NB) cv[c + 1][kk] = cj[K0 + (c + 1) * CH + kk];
      }
#pragma unroll
      for (int kk = 0; kk < CH; ++kk)
        if (K0 + c * CH + kk < NB) a[K0 + c * CH + kk] = fma(-lij, cv[c][kk], a[K0 + c * CH + kk]);
    }
    fs.rinv = rnext;
  }
}

template <typename T, int... Js>
__device__ __forceinline__ void factor_steps(std::integer_sequence<int, Js...>, T (&a)[NB],
                                             FactorState<T>& fs, int nbe, int i, T (*col)[NB],
                                             int z0) {
  (factor_step<T, Js>(a, fs, nbe, i, col, z0), ...);
}

// One column step c of the panel solve X L11^T = M21 (one row per lane):
// x[c] /= L[c][c], then x[k] -= x[c] L[k][c] for k > c, with L[k][c] read from
// lt (row stride NB + 1) in chunks whose reads run ahead of the updates.
template <typename T, int C>
__device__ __forceinline__ void solve_step(T (&x)[NB], const T* ltz, const T* dz) {
  x[C] *= dz[C];
  if constexpr (C + 1 < NB) {
    const T* lc = ltz + C * (NB + 1);
    constexpr int CH = 16, K0 = C + 1, NCH = (NB - K0 + CH - 1) / CH;
    T cv[NCH][CH];
#pragma unroll
    for (int kk = 0; kk < CH; ++kk)
      if (K0 + kk < NB) cv[0][kk] = lc[K0 + kk];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      if (c + 1 < NCH) {
#pragma unroll
        for (int kk = 0; kk < CH; ++kk)
          if (K0 + (c + 1) * CH + kk < NB) cv[c + 1][kk] = lc[K0 + (c + 1) * CH + kk];
      }
#pragma unroll
      for (int kk = 0; kk < CH; ++kk)
        if (K0 + c * CH + kk < NB) x[K0 + c * CH + kk] = fma(-x[C], cv[c][kk], x[K0 + c * CH + kk]);
    }
  }
}

template <typename T, int... Cs>
__device__ __forceinline__ void solve_steps(std::integer_sequence<int, Cs...>, T (&x)[NB],
                                            const T* ltz, const T* dz) {
  (solve_step<T, Cs>(x, ltz, dz), ...);
}

// Workgroup wg of the panel step at column p of an mr x mc lower matrix
// (mr >= mc; rows beyond mc are extra right-hand sides stored as rows, whose
// factor rows come out as L^-1 applied to them): every workgroup factors A11
// from M; wg 0 stores L11 into diag_blk (64 x 64 row-major, lower part) and
// reports the first failing pivot column and the smallest pivot; wg >= 1 also
// solve rows p + nbe + 192 (wg - 1) ... of L21 in place.  L11 goes to the
// side block, not to M, because other workgroups of the same launch may still
// be reading A11 from M; the blocks are copied into M after the last panel.
template <typename T>
__device__ __forceinline__ void potrf_panel_body(int mr, int mc, T* __restrict__ M, long ld, int p,
                                                 int wg, T* __restrict__ diag_blk, int* fail_out,
                                                 unsigned long long* minp_bits_out) {
  __shared__ T col[2][NB];             // column j of L11 (lane i writes row i)
  __shared__ T lt[NB][NB + 1];         // A11 on entry; L11 transposed on exit: lt[c][k] = L[k][c]
  __shared__ T dinv[NB];
  __shared__ T S[kRowsPerWG][NB + 1];  // staged panel rows of this workgroup
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nbe = min(NB, mc - p);
  const bool solve = wg > 0;
  const long r0 = (long)p + nbe + (long)(wg - 1) * kRowsPerWG;

  // stage A11 (identity beyond the matrix; upper part never read) and the
  // workgroup's panel rows, coalesced
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, k = e % NB;
    const T v = M[(long)(p + min(r, nbe - 1)) * ld + p + min(k, nbe - 1)];
    lt[r][k] = (r < nbe && k < nbe) ? v : ((r == k) ? T(1) : T(0));
  }
  if (solve) {
    // columns clamped to the panel (nbe < 64 only in the last panel, whose
    // rows below are extra right-hand-side rows)
    for (int e = tid; e < kRowsPerWG * (NB / 2); e += 256) {
      const int row = e / (NB / 2), kp = 2 * (e % (NB / 2));
      const long gr = min(r0 + row, (long)mr - 1);
      const T* src = M + gr * ld + p;
      S[row][kp] = src[min(kp, nbe - 1)];
      S[row][kp + 1] = src[min(kp + 1, nbe - 1)];
    }
  }
  __syncthreads();

  if (wv == 0) {
    T a[NB];
    const int i = lane;
#pragma unroll
    for (int k = 0; k < NB; ++k) a[k] = lt[i][k];
    const int z0 = opaque_zero();
    T piv = RL<T>::rd(a[0], 0);
    T rinv = RL<T>::rsq(piv);
    FactorState<T> fs{piv, rinv, T(0), T(INFINITY), -1};
    factor_steps<T>(std::make_integer_sequence<int, NB>{}, a, fs, nbe, i, col, z0);
    const int fail = fs.fail;
    const T minp = fs.minp;
    const T myrinv = fs.myrinv;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < NB; ++k) lt[k][i] = a[k];
    dinv[i] = myrinv;
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
      if (r < nbe && k <= r) diag_blk[e] = lt[k][r];
    }
    return;
  }
  if (wv == 0) return;
  const int row = (wv - 1) * 64 + lane;
  const long rr = r0 + row;
  T x[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) x[k] = S[row][k];
  const int z1 = opaque_zero();
  solve_steps<T>(std::make_integer_sequence<int, NB>{}, x, &lt[0][0] + z1, dinv + z1);
  if (rr < mr) {
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k < nbe) M[rr * ld + p + k] = x[k];
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
