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
// one term ahead), so all take the same breakdown decision.  The paper
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
// denominator is reported like a pivot.
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
  double* sa = Ys + (long)(n + 1) * ld;    // a_l, two buffers of m
  const int tid = threadIdx.x;
  for (long e = tid; e < (long)n * m; e += kWbThreads) {
    const long k = e / m, i = e - k * m;
    Ys[k * ld + i] = Y0[e];
  }
  for (int i = tid; i < m; i += kWbThreads) {
    Ys[(long)n * ld + i] = x0[i];
    sa[i] = A[(long)i * n];
  }
  __syncthreads();
  double minden = INFINITY;
  int fail = -1;
  for (int l = 0; l < n; ++l) {
    const double* al = sa + (l & 1) * m;
    if (l + 1 < n)
      for (int i = tid; i < m; i += kWbThreads) sa[((l + 1) & 1) * m + i] = A[(long)i * n + l + 1];
    const double v = d[l] - 1.0;
    if (v != 0.0) {
      const double* yl = Ys + (long)l * ld;
      double dl = 0.0;
      for (int i = 0; i < m; ++i) dl += al[i] * yl[i];
      const double den = 1.0 + v * dl;
      if (!(den > 0.0) || !isfinite(den)) {
        fail = l;  // every thread computed the same den: a uniform exit
        break;
      }
      minden = fmin(minden, den);
      const double f = v / den;
      for (int k = l + 1 + tid; k <= n; k += kWbThreads) {
        double* yk = Ys + (long)k * ld;
        double dk = 0.0;
        for (int i = 0; i < m; ++i) dk += al[i] * yk[i];
        const double ck = f * dk;
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
  return (size_t)((n + 1) * ld + 2 * m) * sizeof(double);
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
