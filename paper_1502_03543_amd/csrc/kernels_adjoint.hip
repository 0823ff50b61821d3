// Reverse mode of one Section 3 step (Section 5 formulas in residual form),
// for a loss on the final iterate.  With the step's own values (r_d, d,
// M = L L^T, dx, dy, ds, g = A^T dy, psi, t, argmax), the chain rule runs
// backwards through
//   x' = x + t dx, y' = y + t dy, s' = s + t ds,   t = alpha_eff / psi,
//   psi = -dx_J/x_J (or -ds_J/s_J) at the argmax J,  dx = -x - d o ds,
//   ds = r_d - g,  g = A^T dy,  M dy = rhs,  M = A D A^T,
//   rhs = b + A (d o r_d),  d = x / s,  r_d = c - A^T y - s.
// The psi == 1 step length is treated as constant.  Each elementwise phase is
// one kernel; the matrix products reuse the forward GEMVs, and the solve with
// M reuses the forward Cholesky factor (M is symmetric).
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ double bsum(double v, double* sh) {
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;
}

// partial sums of xbar.dx + sbar.ds (n) and ybar.dy (m)
__global__ __launch_bounds__(256) void k_tbar_part(long m, long n, const double* xb,
                                                   const double* dx, const double* sb,
                                                   const double* ds, const double* yb,
                                                   const double* dy, double* part) {
  __shared__ double sh[4];
  const long j = blockIdx.x * 256L + threadIdx.x;
  double v = 0;
  if (j < n) v = xb[j] * dx[j] + sb[j] * ds[j];
  if (j < m) v += yb[j] * dy[j];
  const double r = bsum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void k_tbar_final(int nparts, const double* part, double* out) {
  __shared__ double sh[4];
  double v = 0;
  for (int k = threadIdx.x; k < nparts; k += 256) v += part[k];
  const double r = bsum(v, sh);
  if (threadIdx.x == 0) *out = r;
}

// Step, ratio test and dx = -x - d o ds in reverse.
__global__ void k_adj_a(long m, long n, double alpha, const DevInfo* info, const double* tbar,
                        const double* x, const double* s, const double* d, const double* dx,
                        const double* ds, double* xb, double* sb, const double* yb, double* dsb,
                        double* db, double* dyb) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const double psi = info->psi;
  const double aeff = (psi == 1.0) ? 1.0 : alpha;
  const double t = aeff / psi;
  const double psib = -aeff * (*tbar) / (psi * psi);
  const long J = info->argmax;
  if (j < n) {
    double dxb = t * xb[j];
    double dsbj = t * sb[j];
    double xbj = xb[j], sbj = sb[j];
    if (J == j) {
      dxb += -psib / x[j];
      xbj += psib * dx[j] / (x[j] * x[j]);
    } else if (J == n + j) {
      dsbj += -psib / s[j];
      sbj += psib * ds[j] / (s[j] * s[j]);
    }
    xbj -= dxb;
    db[j] = -dxb * ds[j];
    dsbj -= d[j] * dxb;
    xb[j] = xbj;
    sb[j] = sbj;
    dsb[j] = dsbj;
  }
  if (j < m) dyb[j] = t * yb[j];
}

// Everything after lambda = M^-1 dybar, h = A^T lambda (chunk partials P):
// d, rhs and r_d in reverse; the three outer-product factors of Abar.
__global__ void k_adj_b(long m, long n, const double* P, int nchunks, const double* g,
                        const double* rd, const double* d, const double* x, const double* s,
                        const double* lam, const double* dsb, double* db, double* xb, double* sb,
                        double* cb, double* rdb, double* bb, double* v1, double* v2, double* v3) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j < n) {
    double h = 0;
    for (int k = 0; k < nchunks; ++k) h += P[(long)k * n + j];
    double dbj = db[j];
    dbj -= h * g[j];
    dbj += rd[j] * h;
    const double rdbj = dsb[j] + d[j] * h;
    double xbj = xb[j] + dbj / s[j];
    double sbj = sb[j] - dbj * x[j] / (s[j] * s[j]);
    sbj -= rdbj;
    xb[j] = xbj;
    sb[j] = sbj;
    if (cb) cb[j] += rdbj;
    rdb[j] = rdbj;
    db[j] = dbj;
    v1[j] = -dsb[j] - h * d[j];
    v2[j] = d[j] * rd[j] - g[j] * d[j];
    v3[j] = -rdbj;
  }
  if (j < m && bb) bb[j] += lam[j];
}

// Abar (m x n, row-major) += u1 v1^T + u2 v2^T + u3 v3^T
__global__ __launch_bounds__(256) void k_rank3(long m, long n, double* Ab, const double* u1,
                                               const double* v1, const double* u2,
                                               const double* v2, const double* u3,
                                               const double* v3) {
  const long i = blockIdx.y;
  const double a1 = u1[i], a2 = u2[i], a3 = u3[i];
  double* row = Ab + i * n;
  for (long j = blockIdx.x * 256L + threadIdx.x; j < n; j += (long)gridDim.x * 256)
    row[j] += a1 * v1[j] + a2 * v2[j] + a3 * v3[j];
}

__global__ void k_zero(double* p, long count) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

}  // namespace

void launch_zero(hipStream_t st, double* p, long count) {
  if (count <= 0 || !p) return;
  const long blocks = (count + 255) / 256;
  // large buffers: grid-stride is not needed, 1-D grids reach 2^31 blocks
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, p, count);
}

void launch_adj_tbar(hipStream_t st, long m, long n, const double* xb, const double* dx,
                     const double* sb, const double* ds, const double* yb, const double* dy,
                     double* part, double* out) {
  const long len = m > n ? m : n;
  const int nb = cdiv(len, 256);
  hipLaunchKernelGGL(k_tbar_part, dim3(nb), dim3(256), 0, st, m, n, xb, dx, sb, ds, yb, dy, part);
  hipLaunchKernelGGL(k_tbar_final, dim3(1), dim3(256), 0, st, nb, part, out);
}

void launch_adj_a(hipStream_t st, long m, long n, double alpha, const DevInfo* info,
                  const double* tbar, const double* x, const double* s, const double* d,
                  const double* dx, const double* ds, double* xb, double* sb, const double* yb,
                  double* dsb, double* db, double* dyb) {
  const long len = m > n ? m : n;
  hipLaunchKernelGGL(k_adj_a, dim3(cdiv(len, 256)), dim3(256), 0, st, m, n, alpha, info, tbar, x,
                     s, d, dx, ds, xb, sb, yb, dsb, db, dyb);
}

void launch_adj_b(hipStream_t st, long m, long n, const double* P, int nchunks, const double* g,
                  const double* rd, const double* d, const double* x, const double* s,
                  const double* lam, const double* dsb, double* db, double* xb, double* sb,
                  double* cb, double* rdb, double* bb, double* v1, double* v2, double* v3) {
  const long len = m > n ? m : n;
  hipLaunchKernelGGL(k_adj_b, dim3(cdiv(len, 256)), dim3(256), 0, st, m, n, P, nchunks, g, rd, d,
                     x, s, lam, dsb, db, xb, sb, cb, rdb, bb, v1, v2, v3);
}

void launch_rank3(hipStream_t st, long m, long n, double* Ab, const double* u1, const double* v1,
                  const double* u2, const double* v2, const double* u3, const double* v3) {
  const int gx = cdiv(n, 256) < 8 ? cdiv(n, 256) : 8;
  hipLaunchKernelGGL(k_rank3, dim3(gx, m), dim3(256), 0, st, m, n, Ab, u1, v1, u2, v2, u3, v3);
}

}  // namespace pdas
