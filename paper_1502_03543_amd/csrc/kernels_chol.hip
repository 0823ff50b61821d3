// Blocked right-looking Cholesky M = L L^T of the normal matrix (Section 5.1
// names Cholesky as the usual solver for the symmetric positive definite
// A D A^T).  Row-major lower storage, panel width kTB = 64.
//
// Per panel p:
//   1. k_potrf_panel: every workgroup factors the 64 x 64 diagonal block
//      (identical arithmetic in each, so identical results); workgroup 0
//      stores L11, the others each solve one 64-row block of the panel below
//      it, L21 = M21 L11^-T.
//      The diagonal block lives in registers: thread (i, g) owns row i,
//      columns g, g+4, ..., g+60.  Column j is published unscaled through a
//      double-buffered LDS column, so a step needs one barrier.  The panel
//      solve gives each row to a quad of lanes (columns interleaved by 4) and
//      broadcasts finished entries with quad shuffles: no barriers at all.
//      Subtractions run in column order, as in the textbook recurrence.
//   2. trailing update M22 -= L21 L21^T on the matrix cores (the normal-matrix
//      kernel in subtract mode, lower tiles only).
// A pivot that is not a finite positive number is recorded (first column) in
// the iteration info and turns the step into a breakdown; no fallback.
#include <climits>
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

constexpr int NB = kTB;  // 64
constexpr int NC = NB / 4;

// v[idx] for a runtime idx in [0, 16) as a select chain over compile-time
// indices, so the array stays in registers.
#define PDAS_SEL16(v, idx)                                                                  \
  ((idx) == 0 ? (v)[0] : (idx) == 1 ? (v)[1] : (idx) == 2 ? (v)[2] : (idx) == 3 ? (v)[3]   \
   : (idx) == 4 ? (v)[4] : (idx) == 5 ? (v)[5] : (idx) == 6 ? (v)[6] : (idx) == 7 ? (v)[7] \
   : (idx) == 8 ? (v)[8] : (idx) == 9 ? (v)[9] : (idx) == 10 ? (v)[10]                      \
   : (idx) == 11 ? (v)[11] : (idx) == 12 ? (v)[12] : (idx) == 13 ? (v)[13]                  \
   : (idx) == 14 ? (v)[14] : (v)[15])
static_assert(NC == 16, "select chain covers 16 registers");

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_panel(int m, T* __restrict__ M, long ld, int p,
                                                     DevInfo* info) {
  __shared__ T col[2][NB];          // column j of the working block, unscaled
  __shared__ T l[NB][NB + 1];       // finished L11
  __shared__ T dinv[NB];            // 1 / L11[j][j]
  const int tid = threadIdx.x;
  const int nbe = min(NB, m - p);
  const int i = tid & 63, g = tid >> 6;

  // ---- factor the diagonal block (identity-padded beyond nbe) ----
  // Branch-free steps: all operand reads of a step are issued together and
  // masked updates are selects, so LDS latency is paid once per step.
  T a[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int k = g + 4 * c;
    T v = (i == k) ? T(1) : T(0);
    if (i < nbe && k <= i) v = M[(long)(p + i) * ld + p + k];
    a[c] = v;
  }
  if (g == 0) col[0][i] = a[0];
  __syncthreads();
  int fail = -1;
  T minp = T(INFINITY);
  for (int j = 0; j < NB; ++j) {
    const T* cj = col[j & 1];
    T lk[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) lk[c] = cj[g + 4 * c];
    const T piv = cj[j];
    const T ci = cj[i];
    if (tid == 0 && j < nbe) {
      if (fail < 0 && !(piv > T(0) && isfinite(piv))) fail = j;
      if (piv < minp) minp = piv;
    }
    const T ljj = sqrt(piv);
    const T rinv = T(1) / ljj;
    const T li = ci * rinv;
    if (g == 0) {
      if (i > j) l[i][j] = li;
      if (i == j) {
        l[j][j] = ljj;
        dinv[j] = rinv;
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int k = g + 4 * c;
      const T upd = a[c] - li * (lk[c] * rinv);
      a[c] = (k > j && k <= i) ? upd : a[c];
    }
    if (j + 1 < NB && g == ((j + 1) & 3)) col[(j + 1) & 1][i] = PDAS_SEL16(a, (j + 1) >> 2);
    __syncthreads();
  }

  if (blockIdx.x == 0) {
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB, k = e % NB;
      if (r < nbe && k <= r) M[(long)(p + r) * ld + p + k] = l[r][k];
    }
    if (tid == 0) {
      if (fail >= 0) atomicMin(&info->chol_fail, p + fail);
      if (minp < T(INFINITY)) {
        const double mp = minp > T(0) ? (double)minp : 0.0;
        // positive doubles order like their bit patterns
        atomicMin(reinterpret_cast<unsigned long long*>(&info->min_pivot),
                  (unsigned long long)__double_as_longlong(mp));
      }
    }
    return;
  }

  // ---- panel solve for rows r0 .. r0+63: X L11^T = M21 ----
  // Row r belongs to a quad of lanes (q = column mod 4); a finished entry is
  // broadcast with a quad shuffle and subtracted from the later columns.
  const int r0 = p + NB + (blockIdx.x - 1) * NB;
  const int nrow = min(NB, m - r0);
  const int r = tid >> 2, q = tid & 3;
  T x[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c)
    x[c] = (r < nrow) ? M[(long)(r0 + r) * ld + p + q + 4 * c] : T(0);
  const int qbase = (threadIdx.x & 63) & ~3;
  for (int cc = 0; cc < NB; ++cc) {
    const int qo = cc & 3, co = cc >> 2;
    T lk[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) lk[c] = l[q + 4 * c][cc];
    const T xf = __shfl(PDAS_SEL16(x, co) * dinv[cc], qbase + qo, 64);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int k = q + 4 * c;
      const T upd = x[c] - xf * lk[c];
      x[c] = (k == cc) ? xf : ((k > cc) ? upd : x[c]);
    }
  }
  if (r < nrow) {
#pragma unroll
    for (int c = 0; c < NC; ++c) M[(long)(r0 + r) * ld + p + q + 4 * c] = x[c];
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
    hipLaunchKernelGGL(k_potrf_panel<double>, dim3(grid), dim3(256), 0, st, m, M, ld, p, info);
    if (below > 0) {
      const int tile = 64;
      launch_syrk_f64(st, below, NB, M + (long)(p + NB) * ld + p, ld, nullptr,
                      M + (long)(p + NB) * ld + (p + NB), ld, true, tile, 1, nullptr);
    }
  }
}

void launch_potrf_f32(hipStream_t st, int m, float* M, long ld, DevInfo* info) {
  for (int p = 0; p < m; p += NB) {
    const int nbe = (m - p) < NB ? (m - p) : NB;
    const int below = m - p - nbe;
    const int grid = 1 + cdiv(below, NB);
    hipLaunchKernelGGL(k_potrf_panel<float>, dim3(grid), dim3(256), 0, st, m, M, ld, p, info);
    if (below > 0)
      launch_syrk_f32(st, below, NB, M + (long)(p + NB) * ld + p, ld, nullptr,
                      M + (long)(p + NB) * ld + (p + NB), ld, true, 1, nullptr);
  }
}

}  // namespace pdas
