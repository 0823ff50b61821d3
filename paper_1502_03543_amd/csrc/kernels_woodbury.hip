// The paper's own direction solver (Section 5, "Solving (ADA^T)x = b"): only
// D changes between iterations, so A D A^T is split as the constant A A^T
// plus the rank-one terms (d_l - 1) a_l a_l^T, and the Egidi-Maponi
// recurrence applies them one at a time (Sherman-Morrison) to
//   Y = [y_1 | ... | y_n] = (A A^T)^-1 A   and   x = (A A^T)^-1 rhs,
// both computed from a Cholesky factor of A A^T:
//   den_l   = 1 + (d_l - 1) a_l^T y_l,
//   x      -= ((d_l - 1) a_l^T x   / den_l) y_l,
//   y_k    -= ((d_l - 1) a_l^T y_k / den_l) y_l     for k > l,
// and after the n-th term x = (A D A^T)^-1 rhs.  (Readings: x_0 = (AA^T)^-1
// rhs, v_l = (d_l - 1) a_l with D's diagonal indexed by the column, and the
// columns k > l only, since y_l is not needed again.)
//
// The n terms are sequential.  One workgroup keeps Y and x in LDS (column
// k at stride ld, ld odd so that lanes reading their own columns hit
// distinct banks), so each term costs one barrier and no global traffic:
// the workgroup's threads take the columns k > l in turn, and every thread
// forms den_l itself from the broadcast column y_l and a_l (staged in LDS
// in blocks of terms), so all take the same breakdown decision.  The chain
// is bound by LDS instruction issue (about 5m accesses per column and
// term), not by arithmetic.  The paper
// assigns one CUDA block per column and launches a kernel per term; on
// this chip one compute unit running the whole chain avoids n grid-wide
// synchronisations, and the LDS (160 KB) bounds the problem size.
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

constexpr int kWbThreads = 256;

__device__ inline int wb_ld(int m) { return (m & 1) ? m : m + 1; }

// Y0 = L^-T L^-1 A (one thread per column of A, the column written
// contiguously: Y0[k m + i]), L the lower Cholesky factor of A A^T
// (row-major, ld).  Setup only.
__global__ __launch_bounds__(256) void k_wb_cols(int m, int n, const double* __restrict__ L,
                                                 long ld, const double* __restrict__ A,
                                                 double* __restrict__ Y0) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double* y = Y0 + (long)k * m;
  for (int i = 0; i < m; ++i) {
    double acc = A[(long)i * n + k];
    for (int j = 0; j < i; ++j) acc -= L[(long)i * ld + j] * y[j];
    y[i] = acc / L[(long)i * ld + i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double acc = y[i];
    for (int j = i + 1; j < m; ++j) acc -= L[(long)j * ld + i] * y[j];
    y[i] = acc / L[(long)i * ld + i];
  }
}

__global__ void k_wb_fill(long n, double v, double* __restrict__ p) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// The recurrence for one iteration: Y0 (column-major, m x n), x0 (m), d (n)
// in; dy = x_n out.  A term whose denominator is not a finite positive
// number records its index as the breakdown column; the smallest
// denominator is reported like a pivot.  d is staged in LDS once, and the
// columns a_l of A in blocks of kWbBlk terms, so a term waits on no global
// load; the inner products run as four interleaved partial sums (a fixed
// order), which shortens their dependency chains.
constexpr int kWbBlk = 16;

__device__ __forceinline__ double dot4(int m, const double* __restrict__ a,
                                       const double* __restrict__ b) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = 0;
  for (; i + 4 <= m; i += 4) {
    s0 += a[i] * b[i];
    s1 += a[i + 1] * b[i + 1];
    s2 += a[i + 2] * b[i + 2];
    s3 += a[i + 3] * b[i + 3];
  }
  for (; i < m; ++i) s0 += a[i] * b[i];
  return (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(kWbThreads) void k_woodbury(int m, int n,
                                                          const double* __restrict__ A,
                                                          const double* __restrict__ d,
                                                          const double* __restrict__ Y0,
                                                          const double* __restrict__ x0,
                                                          double* __restrict__ dy,
                                                          DevInfo* info) {
  extern __shared__ double lds[];
  const int ld = wb_ld(m);
  double* Ys = lds;                        // n + 1 columns: y_0 .. y_{n-1}, then x
  double* sd = Ys + (long)(n + 1) * ld;    // d
  double* sa = sd + n;                     // a_l of the current block, column l at l % kWbBlk
  const int tid = threadIdx.x;
  for (long e = tid; e < (long)n * m; e += kWbThreads) {
    const long k = e / m, i = e - k * m;
    Ys[k * ld + i] = Y0[e];
  }
  for (int i = tid; i < m; i += kWbThreads) Ys[(long)n * ld + i] = x0[i];
  for (int j = tid; j < n; j += kWbThreads) sd[j] = d[j];
  double minden = INFINITY;
  int fail = -1;
  for (int l = 0; l < n; ++l) {
    if (l % kWbBlk == 0) {
      // the next block of columns of A (the previous block is no longer read:
      // every thread passed the barrier that ended its last term)
      const int nb = min(kWbBlk, n - l);
      for (int e = tid; e < nb * m; e += kWbThreads) {
        const int c = e / m, i = e - c * m;
        sa[c * m + i] = A[(long)i * n + l + c];
      }
      __syncthreads();
    }
    const double* al = sa + (l % kWbBlk) * m;
    const double v = sd[l] - 1.0;
    if (v != 0.0) {
      const double* yl = Ys + (long)l * ld;
      const double den = 1.0 + v * dot4(m, al, yl);
      if (!(den > 0.0) || !isfinite(den)) {
        fail = l;  // every thread computed the same den: a uniform exit
        break;
      }
      minden = fmin(minden, den);
      const double f = v / den;
      for (int k = l + 1 + tid; k <= n; k += kWbThreads) {
        double* yk = Ys + (long)k * ld;
        const double ck = f * dot4(m, al, yk);
        for (int i = 0; i < m; ++i) yk[i] -= ck * yl[i];
      }
    }
    __syncthreads();
  }
  __syncthreads();
  for (int i = tid; i < m; i += kWbThreads) dy[i] = Ys[(long)n * ld + i];
  if (tid == 0) {
    if (fail >= 0) atomicMin(&info->chol_fail, fail);
    if (minden < INFINITY)
      atomicMin(reinterpret_cast<unsigned long long*>(&info->min_pivot),
                (unsigned long long)__double_as_longlong(minden > 0 ? minden : 0.0));
  }
}

}  // namespace

size_t woodbury_lds_bytes(long m, long n) {
  const long ld = (m & 1) ? m : m + 1;
  return (size_t)((n + 1) * ld + n + (long)kWbBlk * m) * sizeof(double);
}

bool woodbury_fits(long m, long n) { return woodbury_lds_bytes(m, n) <= kWoodburyMaxLds; }

hipError_t woodbury_prepare() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_woodbury),
                             hipFuncAttributeMaxDynamicSharedMemorySize, kWoodburyMaxLds);
}

void launch_wb_fill(hipStream_t st, long n, double v, double* p) {
  hipLaunchKernelGGL(k_wb_fill, dim3(cdiv(n, 256)), dim3(256), 0, st, n, v, p);
}

void launch_wb_cols(hipStream_t st, int m, int n, const double* L, long ld, const double* A,
                    double* Y0) {
  hipLaunchKernelGGL(k_wb_cols, dim3(cdiv(n, 256)), dim3(256), 0, st, m, n, L, ld, A, Y0);
}

void launch_woodbury(hipStream_t st, int m, int n, const double* A, const double* d,
                     const double* Y0, const double* x0, double* dy, DevInfo* info) {
  hipLaunchKernelGGL(k_woodbury, dim3(1), dim3(kWbThreads), woodbury_lds_bytes(m, n), st, m, n,
                     A, d, Y0, x0, dy, info);
}

}  // namespace pdas
