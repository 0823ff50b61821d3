// Blocked right-looking Cholesky M = L L^T of the normal matrix (Section 5.1
// names Cholesky as the usual solver for the symmetric positive definite
// A D A^T).  Row-major lower storage, panel width kTB = 64.
//
// Per panel p:
//   1. k_potrf_panel: every workgroup factors the 64 x 64 diagonal block in
//      LDS (identical arithmetic in each, so identical results); workgroup 0
//      stores L11, the others each solve one 64-row block of the panel below
//      it (L21 = M21 L11^-T) with 4 threads per row.
//   2. trailing update M22 -= L21 L21^T on the matrix cores (the normal-matrix
//      kernel in subtract mode, lower tiles only).
// A pivot that is not a finite positive number is recorded (first column) in
// the iteration info and turns the step into a breakdown; no fallback.
#include <climits>
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

constexpr int NB = kTB;

__global__ __launch_bounds__(256) void k_potrf_panel(int m, double* __restrict__ M, long ld,
                                                     int p, DevInfo* info) {
  __shared__ double a[NB][NB + 1];   // working copy of the diagonal block
  __shared__ double l[NB][NB + 1];   // finished L11
  __shared__ double xr[NB][NB + 1];  // this workgroup's rows of the panel
  const int tid = threadIdx.x;
  const int nbe = min(NB, m - p);

  // Load the lower triangle of the diagonal block; pad with the identity.
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e / NB, k = e % NB;
    double v = 0.0;
    if (i < nbe && k <= i) v = M[(long)(p + i) * ld + p + k];
    else if (i == k) v = 1.0;
    a[i][k] = v;
    l[i][k] = 0.0;
  }
  __syncthreads();

  const int i = tid & 63, g = tid >> 6;
  int fail = -1;
  double minp = INFINITY;
  for (int j = 0; j < NB; ++j) {
    const double piv = a[j][j];
    if (j < nbe) {
      if (fail < 0 && !(piv > 0.0 && isfinite(piv))) fail = j;
      if (piv < minp) minp = piv;
    }
    const double ljj = sqrt(piv);
    if (i > j) {
      const double li = a[i][j] / ljj;
      for (int k = j + 1 + g; k <= i; k += 4) a[i][k] -= li * (a[k][j] / ljj);
      if (g == 0) l[i][j] = li;
    } else if (i == j && g == 0) {
      l[j][j] = ljj;
    }
    __syncthreads();
  }

  if (blockIdx.x == 0) {
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB, k = e % NB;
      if (r < nbe && k <= r) M[(long)(p + r) * ld + p + k] = l[r][k];
    }
    if (tid == 0) {
      if (fail >= 0) atomicMin(&info->chol_fail, p + fail);
      if (minp < INFINITY) {
        // positive doubles order like their bit patterns
        atomicMin(reinterpret_cast<unsigned long long*>(&info->min_pivot),
                  (unsigned long long)__double_as_longlong(minp > 0 ? minp : 0.0));
      }
    }
    return;
  }

  // Rows of the panel below the diagonal block handled by this workgroup.
  const int r0 = p + NB + (blockIdx.x - 1) * NB;
  const int nrow = min(NB, m - r0);
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, k = e % NB;
    xr[r][k] = (r < nrow) ? M[(long)(r0 + r) * ld + p + k] : 0.0;
  }
  __syncthreads();
  {
    const int r = tid >> 2, q = tid & 3;
    for (int c = 0; c < NB; ++c) {
      const double mv = xr[r][c];
      double part = 0.0;
      for (int k = q; k < c; k += 4) part += xr[r][k] * l[c][k];
      part += __shfl_xor(part, 1, 64);
      part += __shfl_xor(part, 2, 64);
      const double v = (mv - part) / l[c][c];
      if ((c & 3) == q) xr[r][c] = v;
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, k = e % NB;
    if (r < nrow) M[(long)(r0 + r) * ld + p + k] = xr[r][k];
  }
}

}  // namespace

void launch_potrf_f64(hipStream_t st, int m, double* M, long ld, DevInfo* info, double* part,
                      size_t part_elems) {
  (void)part;
  (void)part_elems;
  for (int p = 0; p < m; p += NB) {
    const int nbe = (m - p) < NB ? (m - p) : NB;
    const int below = m - p - nbe;
    const int grid = 1 + cdiv(below, NB);
    hipLaunchKernelGGL(k_potrf_panel, dim3(grid), dim3(256), 0, st, m, M, ld, p, info);
    if (below > 0) {
      const int tile = below >= 2048 ? 128 : 64;
      launch_syrk_f64(st, below, NB, M + (long)(p + NB) * ld + p, ld, nullptr,
                      M + (long)(p + NB) * ld + (p + NB), ld, true, tile, 1, nullptr);
    }
  }
}

}  // namespace pdas
