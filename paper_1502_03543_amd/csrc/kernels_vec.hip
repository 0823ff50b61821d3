// Bandwidth-bound kernels of one PDAS iteration: residuals, GEMVs over A,
// the direction / ratio test and the step (Section 3 algorithm; Section 5
// component formulas in residual form).  Every reduction runs in a fixed
// order (per-block trees, then an ordered pass over block partials), so the
// results are bitwise reproducible run to run.
#include <climits>
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

constexpr int kT = kVecThreads;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum with a fixed tree; result valid in thread 0.
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// (value, index) max with the smallest index among equal values.
__device__ inline void argmax_merge(double& v, long long& i, double v2, long long i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

__device__ void block_argmax(double& v, long long& i, double* shv, long long* shi) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    double v2 = __shfl_xor(v, o, 64);
    long long i2 = __shfl_xor(i, o, 64);
    argmax_merge(v, i, v2, i2);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    shv[w] = v;
    shi[w] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int k = 1; k < nw; ++k) argmax_merge(v, i, shv[k], shi[k]);
  }
  __syncthreads();
}

__global__ void k_check_inputs(long m, long n, const double* A, const double* b,
                               const double* c, const double* x, const double* y,
                               const double* s, DevCheck* chk) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long stride = (long)gridDim.x * blockDim.x;
  int bad = 0, nonpos = 0;
  if (A)  // a CSR A is checked by its own kernel
    for (long i = tid; i < m * n; i += stride) bad |= !isfinite(A[i]);
  for (long i = tid; i < m; i += stride) bad |= !isfinite(b[i]) | !isfinite(y[i]);
  for (long i = tid; i < n; i += stride) {
    bad |= !isfinite(c[i]) | !isfinite(x[i]) | !isfinite(s[i]);
    nonpos |= !(x[i] > 0) | !(s[i] > 0);
  }
  if (bad) atomicOr(&chk->nonfinite, 1);
  if (nonpos) atomicOr(&chk->nonpos, 1);
}

__global__ void k_fill_i32(int* p, int v, long count) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void k_iter_begin(DevInfo* info, int* sync, int nsync) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    info->status = LP_OK;
    info->chol_fail = INT_MAX;
    info->min_pivot = INFINITY;
    info->zero_dir = 0;
    info->trsv_err = 0;
    info->lost = 0;
    info->nonfinite = 0;
    info->refine_steps = 0;
    info->refine_resid = 0.0;
  }
  for (int i = tid; i < nsync; i += blockDim.x) sync[i] = 0;
}

// r_d = c - sum_chunks P[chunk][j] - s  (Section 3 KKT row A^T y + s = c).
__global__ void k_dual_resid(long n, const double* P, int nchunks, const double* c,
                             const double* s, double* rd) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= n) return;
  double g = 0;
  for (int k = 0; k < nchunks; ++k) g += P[(long)k * n + j];
  rd[j] = c[j] - g - s[j];
}

// D = S^-1 X (Section 5) and w = d o r_d; sd = sqrt(d) in FP32 when asked
// (the column scaling of the FP32 normal matrix).
__global__ void k_prep(long n, const double* x, const double* s, const double* rd, double* d,
                       double* w, float* sd) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double dj = x[j] / s[j];
  d[j] = dj;
  w[j] = dj * rd[j];
  if (sd) sd[j] = (float)sqrt(dj);
}

// out = b + sign * A w, one wavefront per row of the row-major A.
__global__ __launch_bounds__(256) void k_gemv_n(long m, long n, const double* __restrict__ A,
                                                const double* __restrict__ w,
                                                const double* __restrict__ b, double sign,
                                                double* out) {
  const long row = blockIdx.x * 4L + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;
  const double* a = A + row * n;
  double acc = 0;
  if ((n & 1) == 0 && ((((uintptr_t)A) | ((uintptr_t)w)) & 15) == 0) {
    const double2* a2 = reinterpret_cast<const double2*>(a);
    const double2* w2 = reinterpret_cast<const double2*>(w);
    const long n2 = n >> 1;
#pragma unroll 8
    for (long j = lane; j < n2; j += 64) {
      const double2 av = a2[j], wv = w2[j];
      acc += av.x * wv.x;
      acc += av.y * wv.y;
    }
  } else {
    for (long j = lane; j < n; j += 64) acc += a[j] * w[j];
  }
  acc = wave_sum(acc);
  if (lane == 0) out[row] = b[row] + sign * acc;
}

// Partial transposed products over chunks of kGemvRows rows:
//   P1[chunk][j] = sum_{i in chunk} A_ij v1_i   (and P2 with v2 when given).
__global__ __launch_bounds__(256) void k_gemv_t(long m, long n, const double* __restrict__ A,
                                                const double* __restrict__ v1,
                                                const double* __restrict__ v2, double* P1,
                                                double* P2) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long chunk = blockIdx.y;
  __shared__ double sv1[kGemvRows], sv2[kGemvRows];
  const long i0 = chunk * kGemvRows;
  const long i1 = min(m, i0 + kGemvRows);
  if (threadIdx.x < i1 - i0) {
    sv1[threadIdx.x] = v1[i0 + threadIdx.x];
    if (v2) sv2[threadIdx.x] = v2[i0 + threadIdx.x];
  }
  __syncthreads();
  if (j >= n) return;
  double a1 = 0, a2 = 0;
  const double* a = A + i0 * n + j;
  // (unrolled: the row loads run ahead of the sequential accumulation)
  if (v2) {
#pragma unroll 16
    for (long i = 0; i < i1 - i0; ++i) {
      const double av = a[i * n];
      a1 += av * sv1[i];
      a2 += av * sv2[i];
    }
    P2[chunk * n + j] = a2;
  } else {
#pragma unroll 16
    for (long i = 0; i < i1 - i0; ++i) a1 += a[i * n] * sv1[i];
  }
  P1[chunk * n + j] = a1;
}

// Direction and per-block ratio test (Section 3 psi, Section 5 formulas):
//   g = A^T dy, ds = r_d - g, dx = -x - d o ds,
//   u_j = -dx_j/x_j (index j), v_j = -ds_j/s_j (index n + j).
__global__ __launch_bounds__(256) void k_dir(long n, const double* P1, const double* P2,
                                             int nchunks, const double* rd, const double* x,
                                             const double* s, const double* d, double* dx,
                                             double* ds, double* gy, double* gout,
                                             double* rpart, long long* ipart, int* zpart,
                                             int* npart) {
  __shared__ double shv[4];
  __shared__ long long shi[4];
  __shared__ int shz, shn;
  if (threadIdx.x == 0) {
    shz = 0;
    shn = 0;
  }
  __syncthreads();
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  double best = -INFINITY;
  long long bi = LLONG_MAX;
  int nz = 0, nf = 0;
  if (j < n) {
    // the chunk partials in chunk order; unrolled so that the loads are
    // issued ahead of the (still sequential) additions
    double g = 0, gyv = 0;
#pragma unroll 8
    for (int k = 0; k < nchunks; ++k) g += P1[(long)k * n + j];
    if (P2) {
#pragma unroll 8
      for (int k = 0; k < nchunks; ++k) gyv += P2[(long)k * n + j];
      gy[j] = gyv;
    }
    gout[j] = g;
    const double dsj = rd[j] - g;
    const double dxj = -x[j] - d[j] * dsj;
    ds[j] = dsj;
    dx[j] = dxj;
    const double u = -dxj / x[j];
    const double v = -dsj / s[j];
    nz = (dxj != 0.0) | (dsj != 0.0);
    nf = !isfinite(u) | !isfinite(v);
    best = u;
    bi = j;
    argmax_merge(best, bi, v, n + j);
  }
  if (nz) atomicOr(&shz, 1);
  if (nf) atomicOr(&shn, 1);
  block_argmax(best, bi, shv, shi);
  if (threadIdx.x == 0) {
    rpart[blockIdx.x] = best;
    ipart[blockIdx.x] = bi;
    zpart[blockIdx.x] = shz;
    npart[blockIdx.x] = shn;
  }
}

// Ratio-test reduction (every block, same order), psi == 1 rule and step.
__global__ __launch_bounds__(256) void k_step(long m, long n, double alpha, int nparts,
                                              const double* rpart, const long long* ipart,
                                              const int* zpart, const int* npart,
                                              const double* dy, const double* x,
                                              const double* y, const double* s,
                                              const double* dx, const double* ds,
                                              const double* g, const double* gy,
                                              const double* c, double* xn, double* yn,
                                              double* sn, double* rdn, double* gap_part,
                                              int* lost_part, DevInfo* info) {
  __shared__ double s_psi;
  __shared__ long long s_arg;
  __shared__ int s_zero, s_nf, s_dyz;
  __shared__ double sh[4];
  __shared__ int s_lost;
  if (threadIdx.x == 0) {
    double p = rpart[0];
    long long a = ipart[0];
    int z = zpart[0], nf = npart[0];
    for (int k = 1; k < nparts; ++k) {
      argmax_merge(p, a, rpart[k], ipart[k]);
      z |= zpart[k];
      nf |= npart[k];
    }
    s_psi = p;
    s_arg = a;
    s_zero = !z;
    s_nf = nf;
    s_dyz = 0;
    s_lost = 0;
  }
  __syncthreads();
  // Zero-direction stop needs dy too (only examined when dx = ds = 0).
  if (s_zero) {
    int nzy = 0;
    for (long i = threadIdx.x; i < m; i += blockDim.x) nzy |= (dy[i] != 0.0);
    if (nzy) atomicOr(&s_dyz, 1);
    __syncthreads();
  }
  const bool zero_dir = s_zero && !s_dyz;
  const double psi = s_psi;
  const bool broke = info->chol_fail != INT_MAX || info->trsv_err != 0;
  const bool bad_psi = s_nf || !(psi > 0) || !isfinite(psi);
  const bool update = !broke && !zero_dir && !bad_psi;
  const double aeff = (psi == 1.0) ? 1.0 : alpha;
  const double t = aeff / psi;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  double gp = 0;
  int lost = 0;
  if (update) {
    if (i < n) {
      const double xv = x[i] + t * dx[i];
      const double sv = s[i] + t * ds[i];
      xn[i] = xv;
      sn[i] = sv;
      rdn[i] = c[i] - (gy[i] + t * g[i]) - sv;
      gp = xv * sv;
      lost = !(xv > 0) | !(sv > 0);
    }
    if (i < m) yn[i] = y[i] + t * dy[i];
  }
  if (lost) atomicOr(&s_lost, 1);
  const double bs = block_sum(gp, sh);
  if (threadIdx.x == 0) {
    gap_part[blockIdx.x] = bs;
    lost_part[blockIdx.x] = s_lost;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    info->psi = psi;
    info->argmax = s_arg;
    info->t = update ? t : 0.0;
    info->zero_dir = zero_dir;
    info->nonfinite = s_nf;
    int st = LP_OK;
    if (info->trsv_err) st = LP_ERR_DEVICE;
    else if (info->chol_fail != INT_MAX) st = LP_ERR_BREAKDOWN;
    else if (zero_dir) st = LP_OPTIMAL_ZERO_DIR;
    else if (bad_psi) st = LP_ERR_NONPOS_PSI;
    info->status = st;
  }
}

// Final status and the new gap (ordered sum of block partials).
__global__ __launch_bounds__(256) void k_finish(int nparts, const double* gap_part,
                                                const int* lost_part, DevInfo* info) {
  __shared__ double sh[4];
  __shared__ int s_lost;
  if (threadIdx.x == 0) s_lost = 0;
  __syncthreads();
  double v = 0;
  int l = 0;
  for (int k = threadIdx.x; k < nparts; k += blockDim.x) {
    v += gap_part[k];
    l |= lost_part[k];
  }
  if (l) atomicOr(&s_lost, 1);
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) {
    int st = info->status;
    if (st == LP_OK) {
      info->gap_after = tot;
      if (info->psi == 1.0) st = LP_OPTIMAL_PSI1;
      else if (s_lost) st = LP_ERR_LOST_INTERIOR;
    }
    info->lost = s_lost;
    info->status = st;
  }
}

__global__ __launch_bounds__(256) void k_gap_part(long n, const double* x, const double* s,
                                                  double* part) {
  __shared__ double sh[4];
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const double v = (j < n) ? x[j] * s[j] : 0.0;
  const double bs = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

__global__ __launch_bounds__(256) void k_gap_final(int nparts, const double* part, double* out) {
  __shared__ double sh[4];
  double v = 0;
  for (int k = threadIdx.x; k < nparts; k += blockDim.x) v += part[k];
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) *out = tot;
}

__global__ void k_copy(double* dst, const double* src, long count) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

// ---- mixed precision helpers ----------------------------------------------

__global__ void k_to_f32(long count, const double* __restrict__ src, float* __restrict__ dst) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < count) dst[i] = (float)src[i];
}

// Squared column norms of A (once at setup): c_j = sum_i A_ij^2, so that
// trace(A D A^T) = sum_j d_j c_j.
__global__ __launch_bounds__(256) void k_colsq(long m, long n, const double* __restrict__ A,
                                               double* out) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= n) return;
  double acc = 0;
  for (long i = 0; i < m; ++i) {
    const double a = A[i * n + j];
    acc += a * a;
  }
  out[j] = acc;
}

// v_j = d_j * sum_chunks P[chunk][j]  (d o A^T dy for the matrix-free residual)
__global__ void k_scale_partials(long n, const double* P, int nchunks, const double* d,
                                 double* v) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= n) return;
  double g = 0;
  for (int k = 0; k < nchunks; ++k) g += P[(long)k * n + j];
  v[j] = d[j] * g;
}

__global__ void k_axpy(long count, const double* __restrict__ x, double* __restrict__ y) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < count) y[i] += x[i];
}

// Refinement test quantities: out[0] = ||r||_inf, out[1] = ||dy||_inf,
// out[2] = trace(M) = sum_j d_j c_j (one workgroup, fixed order).
__global__ __launch_bounds__(256) void k_refine_norms(long m, long n, const double* r,
                                                      const double* dy, const double* d,
                                                      const double* colsq, double* out) {
  __shared__ double sh[4];
  __shared__ double smax[2][4];
  double rn = 0, yn = 0, tr = 0;
  for (long i = threadIdx.x; i < m; i += blockDim.x) {
    rn = fmax(rn, fabs(r[i]));
    yn = fmax(yn, fabs(dy[i]));
  }
  for (long j = threadIdx.x; j < n; j += blockDim.x) tr += d[j] * colsq[j];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    rn = fmax(rn, __shfl_xor(rn, o, 64));
    yn = fmax(yn, __shfl_xor(yn, o, 64));
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    smax[0][w] = rn;
    smax[1][w] = yn;
  }
  const double t = block_sum(tr, sh);
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      a = fmax(a, smax[0][k]);
      b = fmax(b, smax[1][k]);
    }
    out[0] = a;
    out[1] = b;
    out[2] = t;
  }
}

// FP32 factor (row-major lower, ld32) widened into the FP64 buffer (ld64).
__global__ void k_lower_f32_to_f64(long m, const float* __restrict__ L32, long ld32,
                                   double* __restrict__ L64, long ld64) {
  const long i = blockIdx.y;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j <= i; j += (long)gridDim.x * blockDim.x)
    L64[i * ld64 + j] = (double)L32[i * ld32 + j];
}

// ---- predictor-corrector (Mehrotra) ---------------------------------------
// The method the previous-work section cites: the affine-scaling (Section 3)
// direction as predictor, a centring parameter from its step, and a second
// solve with the same factor whose third right-hand side carries the
// second-order term dX_aff dS_aff e and the centring target sigma mu e;
// primal and dual steps are eta times the step to the boundary, capped at 1.

// Block minimum; result valid in thread 0.
__device__ double block_min(double v, double* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = INFINITY;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) r = fmin(r, sh[i]);
  }
  __syncthreads();
  return r;
}

// Steps to the boundary from the per-block minima (every block reduces the
// same partials, so every block holds the same value): thread 0's result.
__device__ void reduce_steps(int nparts, const double* amin, double* s_ap, double* s_ad) {
  if (threadIdx.x == 0) {
    double ap = INFINITY, ad = INFINITY;
    for (int k = 0; k < nparts; ++k) {
      ap = fmin(ap, amin[2 * k]);
      ad = fmin(ad, amin[2 * k + 1]);
    }
    *s_ap = ap;
    *s_ad = ad;
  }
  __syncthreads();
}

// Predictor: g = A^T dy_aff, g_y = A^T y (chunk partials, in chunk order),
// ds_aff = r_d - g, dx_aff = -x - d o ds_aff, and per block the steps to
// the boundary min over dx_j < 0 of -x_j/dx_j (and for s, ds).
__global__ __launch_bounds__(256) void k_pc_aff(long n, const double* P1, const double* P2,
                                                int nchunks, const double* rd, const double* x,
                                                const double* s, const double* d, double* dxa,
                                                double* dsa, double* gy, double* amin) {
  __shared__ double sh[4];
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  double rp = INFINITY, rq = INFINITY;
  if (j < n) {
    double g = 0, gyv = 0;
#pragma unroll 8
    for (int k = 0; k < nchunks; ++k) g += P1[(long)k * n + j];
#pragma unroll 8
    for (int k = 0; k < nchunks; ++k) gyv += P2[(long)k * n + j];
    gy[j] = gyv;
    const double dsj = rd[j] - g;
    const double dxj = -x[j] - d[j] * dsj;
    dsa[j] = dsj;
    dxa[j] = dxj;
    if (dxj < 0) rp = -x[j] / dxj;
    if (dsj < 0) rq = -s[j] / dsj;
  }
  const double bp = block_min(rp, sh);
  const double bq = block_min(rq, sh);
  if (threadIdx.x == 0) {
    amin[2 * blockIdx.x] = bp;
    amin[2 * blockIdx.x + 1] = bq;
  }
}

// mu_aff partials: per block, sum of (x + a_p dx_aff)(s + a_d ds_aff) with
// the predictor steps a = min(1, step to the boundary).
__global__ __launch_bounds__(256) void k_pc_mu(long n, int nparts, const double* amin,
                                               const double* x, const double* s,
                                               const double* dxa, const double* dsa,
                                               double* mupart) {
  __shared__ double sh[4];
  __shared__ double s_ap, s_ad;
  reduce_steps(nparts, amin, &s_ap, &s_ad);
  const double ap = fmin(1.0, s_ap), ad = fmin(1.0, s_ad);
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const double v = (j < n) ? (x[j] + ap * dxa[j]) * (s[j] + ad * dsa[j]) : 0.0;
  const double bs = block_sum(v, sh);
  if (threadIdx.x == 0) mupart[blockIdx.x] = bs;
}

// Centring sigma = (mu_aff / mu)^3 with mu = gap / n; the corrector's
// column term q = (dx_aff o ds_aff - sigma mu) / s and w = d o r_d + q, so
// that the corrector's reduced right-hand side is b + A w and its
// dx = -x - q - d o ds.
__global__ __launch_bounds__(256) void k_pc_corr(long n, int nparts, const double* mupart,
                                                 const double* amin, double gap,
                                                 const double* rd, const double* s,
                                                 const double* d, const double* dxa,
                                                 const double* dsa, double* q, double* w,
                                                 DevInfo* info) {
  __shared__ double s_sig;
  if (threadIdx.x == 0) {
    double acc = 0;
    for (int k = 0; k < nparts; ++k) acc += mupart[k];
    const double mu = gap / (double)n, r = (acc / (double)n) / mu;
    s_sig = r * r * r;
    if (blockIdx.x == 0) {
      double ap = INFINITY, ad = INFINITY;
      for (int k = 0; k < nparts; ++k) {
        ap = fmin(ap, amin[2 * k]);
        ad = fmin(ad, amin[2 * k + 1]);
      }
      info->sigma = s_sig;
      info->mu_aff = acc / (double)n;
      info->alpha_aff_p = fmin(1.0, ap);
      info->alpha_aff_d = fmin(1.0, ad);
    }
  }
  __syncthreads();
  const double smu = s_sig * (gap / (double)n);
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double qj = (dxa[j] * dsa[j] - smu) / s[j];
  q[j] = qj;
  w[j] = d[j] * rd[j] + qj;
}

// Corrector direction: g = A^T dy, ds = r_d - g, dx = -x - q - d o ds, the
// per-block steps to the boundary and the zero / non-finite flags.
__global__ __launch_bounds__(256) void k_pc_dir(long n, const double* P1, int nchunks,
                                                const double* rd, const double* x,
                                                const double* s, const double* d,
                                                const double* q, double* dx, double* ds,
                                                double* gout, double* amin, int* zpart,
                                                int* npart) {
  __shared__ double sh[4];
  __shared__ int shz, shn;
  if (threadIdx.x == 0) {
    shz = 0;
    shn = 0;
  }
  __syncthreads();
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  double rp = INFINITY, rq = INFINITY;
  int nz = 0, nf = 0;
  if (j < n) {
    double g = 0;
#pragma unroll 8
    for (int k = 0; k < nchunks; ++k) g += P1[(long)k * n + j];
    gout[j] = g;
    const double dsj = rd[j] - g;
    const double dxj = -x[j] - q[j] - d[j] * dsj;
    ds[j] = dsj;
    dx[j] = dxj;
    if (dxj < 0) rp = -x[j] / dxj;
    if (dsj < 0) rq = -s[j] / dsj;
    nz = (dxj != 0.0) | (dsj != 0.0);
    nf = !isfinite(dxj) | !isfinite(dsj);
  }
  if (nz) atomicOr(&shz, 1);
  if (nf) atomicOr(&shn, 1);
  const double bp = block_min(rp, sh);
  const double bq = block_min(rq, sh);
  if (threadIdx.x == 0) {
    amin[2 * blockIdx.x] = bp;
    amin[2 * blockIdx.x + 1] = bq;
    zpart[blockIdx.x] = shz;
    npart[blockIdx.x] = shn;
  }
}

// Corrector step: a_p = min(1, eta a_max_p), a_d = min(1, eta a_max_d);
// x += a_p dx, y += a_d dy, s += a_d ds; next r_d = c - (A^T y + a_d A^T dy)
// - s; gap partials; statuses as for the Section 3 step (no psi == 1 rule).
__global__ __launch_bounds__(256) void k_pc_step(long m, long n, double eta, int nparts,
                                                 const double* amin, const int* zpart,
                                                 const int* npart, const double* dy,
                                                 const double* x, const double* y,
                                                 const double* s, const double* dx,
                                                 const double* ds, const double* g,
                                                 const double* gy, const double* c, double* xn,
                                                 double* yn, double* sn, double* rdn,
                                                 double* gap_part, int* lost_part,
                                                 DevInfo* info) {
  __shared__ double s_ap, s_ad;
  __shared__ int s_zero, s_nf, s_dyz, s_lost;
  __shared__ double sh[4];
  if (threadIdx.x == 0) {
    double ap = INFINITY, ad = INFINITY;
    int z = 0, nf = 0;
    for (int k = 0; k < nparts; ++k) {
      ap = fmin(ap, amin[2 * k]);
      ad = fmin(ad, amin[2 * k + 1]);
      z |= zpart[k];
      nf |= npart[k];
    }
    s_ap = fmin(1.0, eta * ap);
    s_ad = fmin(1.0, eta * ad);
    s_zero = !z;
    s_nf = nf;
    s_dyz = 0;
    s_lost = 0;
  }
  __syncthreads();
  if (s_zero) {
    int nzy = 0;
    for (long i = threadIdx.x; i < m; i += blockDim.x) nzy |= (dy[i] != 0.0);
    if (nzy) atomicOr(&s_dyz, 1);
    __syncthreads();
  }
  const bool zero_dir = s_zero && !s_dyz;
  const double ap = s_ap, ad = s_ad;
  const bool broke = info->chol_fail != INT_MAX || info->trsv_err != 0;
  const bool bad = s_nf || !(ap > 0) || !(ad > 0) || !isfinite(ap) || !isfinite(ad);
  const bool update = !broke && !zero_dir && !bad;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  double gp = 0;
  int lost = 0;
  if (update) {
    if (i < n) {
      const double xv = x[i] + ap * dx[i];
      const double sv = s[i] + ad * ds[i];
      xn[i] = xv;
      sn[i] = sv;
      rdn[i] = c[i] - (gy[i] + ad * g[i]) - sv;
      gp = xv * sv;
      lost = !(xv > 0) | !(sv > 0);
    }
    if (i < m) yn[i] = y[i] + ad * dy[i];
  }
  if (lost) atomicOr(&s_lost, 1);
  const double bs = block_sum(gp, sh);
  if (threadIdx.x == 0) {
    gap_part[blockIdx.x] = bs;
    lost_part[blockIdx.x] = s_lost;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    info->psi = NAN;  // no ratio-test value in this method
    info->argmax = -1;
    info->alpha_p = update ? ap : 0.0;
    info->alpha_d = update ? ad : 0.0;
    info->t = info->alpha_p;
    info->zero_dir = zero_dir;
    info->nonfinite = s_nf;
    int st = LP_OK;
    if (info->trsv_err) st = LP_ERR_DEVICE;
    else if (info->chol_fail != INT_MAX) st = LP_ERR_BREAKDOWN;
    else if (zero_dir) st = LP_OPTIMAL_ZERO_DIR;
    else if (bad) st = LP_ERR_NONPOS_PSI;
    info->status = st;
  }
}

}  // namespace

void launch_pc_aff(hipStream_t st, long n, const double* P1, const double* P2, int nchunks,
                   const double* rd, const double* x, const double* s, const double* d,
                   double* dxa, double* dsa, double* gy, double* amin) {
  hipLaunchKernelGGL(k_pc_aff, dim3(dir_blocks(n)), dim3(256), 0, st, n, P1, P2, nchunks, rd, x,
                     s, d, dxa, dsa, gy, amin);
}

void launch_pc_corr(hipStream_t st, long n, double gap, const double* amin, const double* x,
                    const double* s, const double* rd, const double* d, const double* dxa,
                    const double* dsa, double* mupart, double* q, double* w, DevInfo* info) {
  const int nb = dir_blocks(n);
  hipLaunchKernelGGL(k_pc_mu, dim3(nb), dim3(256), 0, st, n, nb, amin, x, s, dxa, dsa, mupart);
  hipLaunchKernelGGL(k_pc_corr, dim3(nb), dim3(256), 0, st, n, nb, mupart, amin, gap, rd, s, d,
                     dxa, dsa, q, w, info);
}

void launch_pc_dir(hipStream_t st, long n, const double* P1, int nchunks, const double* rd,
                   const double* x, const double* s, const double* d, const double* q,
                   double* dx, double* ds, double* g, double* amin, int* zpart, int* npart) {
  hipLaunchKernelGGL(k_pc_dir, dim3(dir_blocks(n)), dim3(256), 0, st, n, P1, nchunks, rd, x, s,
                     d, q, dx, ds, g, amin, zpart, npart);
}

void launch_pc_step(hipStream_t st, long m, long n, double eta, const double* amin,
                    const int* zpart, const int* npart, const double* dy, const double* x,
                    const double* y, const double* s, const double* dx, const double* ds,
                    const double* g, const double* gy, const double* c, double* xn, double* yn,
                    double* sn, double* rdn, double* gap_part, int* lost_part, DevInfo* info) {
  hipLaunchKernelGGL(k_pc_step, dim3(step_blocks(m, n)), dim3(256), 0, st, m, n, eta,
                     dir_blocks(n), amin, zpart, npart, dy, x, y, s, dx, ds, g, gy, c, xn, yn,
                     sn, rdn, gap_part, lost_part, info);
}

void launch_check_inputs(hipStream_t st, long m, long n, const double* A, const double* b,
                         const double* c, const double* x, const double* y, const double* s,
                         DevCheck* chk) {
  long work = m * n > n ? m * n : n;
  int blocks = cdiv(work, kT);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_check_inputs, dim3(blocks), dim3(kT), 0, st, m, n, A, b, c, x, y, s, chk);
}

void launch_fill_i32(hipStream_t st, int* p, int v, long count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(count, kT)), dim3(kT), 0, st, p, v, count);
}

void launch_iter_begin(hipStream_t st, DevInfo* info, int* trsv_sync, int nblk) {
  hipLaunchKernelGGL(k_iter_begin, dim3(1), dim3(kT), 0, st, info, trsv_sync, 4 + 2 * nblk);
}

void launch_dual_resid(hipStream_t st, long m, long n, const double* P, int nchunks,
                       const double* c, const double* s, double* rd) {
  (void)m;
  hipLaunchKernelGGL(k_dual_resid, dim3(cdiv(n, kT)), dim3(kT), 0, st, n, P, nchunks, c, s, rd);
}

void launch_prep(hipStream_t st, long n, const double* x, const double* s, const double* rd,
                 double* d, double* w, float* sd) {
  hipLaunchKernelGGL(k_prep, dim3(cdiv(n, kT)), dim3(kT), 0, st, n, x, s, rd, d, w, sd);
}

void launch_gemv_n(hipStream_t st, long m, long n, const double* A, const double* w,
                   const double* b, double* out, double sign) {
  hipLaunchKernelGGL(k_gemv_n, dim3(cdiv(m, 4)), dim3(256), 0, st, m, n, A, w, b, sign, out);
}

int gemv_t_chunks(long m) { return cdiv(m, kGemvRows); }

void launch_gemv_t(hipStream_t st, long m, long n, const double* A, const double* v1,
                   const double* v2, double* P1, double* P2) {
  hipLaunchKernelGGL(k_gemv_t, dim3(cdiv(n, 256), gemv_t_chunks(m)), dim3(256), 0, st, m, n, A,
                     v1, v2, P1, P2);
}

int dir_blocks(long n) { return cdiv(n, 256); }

void launch_dir(hipStream_t st, long m, long n, const double* P1, const double* P2, int nchunks,
                const double* rd, const double* x, const double* s, const double* d,
                double* dx, double* ds, double* gy, double* g, double* rpart, long long* ipart,
                int* zpart, int* npart) {
  (void)m;
  hipLaunchKernelGGL(k_dir, dim3(dir_blocks(n)), dim3(256), 0, st, n, P1, P2, nchunks, rd, x, s,
                     d, dx, ds, gy, g, rpart, ipart, zpart, npart);
}

int step_blocks(long m, long n) { return cdiv(m > n ? m : n, 256); }

void launch_step(hipStream_t st, long m, long n, double alpha, int nparts, const double* rpart,
                 const long long* ipart, const int* zpart, const int* npart, const double* dy,
                 const double* x, const double* y, const double* s, const double* dx,
                 const double* ds, const double* g, const double* gy, const double* c,
                 double* xn, double* yn, double* sn, double* rdn, double* gap_part,
                 int* lost_part, DevInfo* info) {
  hipLaunchKernelGGL(k_step, dim3(step_blocks(m, n)), dim3(256), 0, st, m, n, alpha, nparts,
                     rpart, ipart, zpart, npart, dy, x, y, s, dx, ds, g, gy, c, xn, yn, sn, rdn,
                     gap_part, lost_part, info);
}

void launch_finish(hipStream_t st, int nparts, const double* gap_part, const int* lost_part,
                   DevInfo* info) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, st, nparts, gap_part, lost_part, info);
}

void launch_gap(hipStream_t st, long n, const double* x, const double* s, double* gap_part,
                double* out) {
  const int nb = cdiv(n, 256);
  hipLaunchKernelGGL(k_gap_part, dim3(nb), dim3(256), 0, st, n, x, s, gap_part);
  hipLaunchKernelGGL(k_gap_final, dim3(1), dim3(256), 0, st, nb, gap_part, out);
}

void launch_copy(hipStream_t st, double* dst, const double* src, long count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3(cdiv(count, kT)), dim3(kT), 0, st, dst, src, count);
}

void launch_to_f32(hipStream_t st, long count, const double* src, float* dst) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_to_f32, dim3(cdiv(count, kT)), dim3(kT), 0, st, count, src, dst);
}

void launch_colsq(hipStream_t st, long m, long n, const double* A, double* out) {
  hipLaunchKernelGGL(k_colsq, dim3(cdiv(n, 256)), dim3(256), 0, st, m, n, A, out);
}

void launch_scale_partials(hipStream_t st, long n, const double* P, int nchunks, const double* d,
                           double* v) {
  hipLaunchKernelGGL(k_scale_partials, dim3(cdiv(n, kT)), dim3(kT), 0, st, n, P, nchunks, d, v);
}

void launch_axpy(hipStream_t st, long count, const double* x, double* y) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_axpy, dim3(cdiv(count, kT)), dim3(kT), 0, st, count, x, y);
}

void launch_refine_norms(hipStream_t st, long m, long n, const double* r, const double* dy,
                         const double* d, const double* colsq, double* out) {
  hipLaunchKernelGGL(k_refine_norms, dim3(1), dim3(256), 0, st, m, n, r, dy, d, colsq, out);
}

void launch_lower_f32_to_f64(hipStream_t st, long m, const float* L32, long ld32, double* L64,
                             long ld64) {
  const int bx = m > 256 ? cdiv(m, 256) : 1;
  hipLaunchKernelGGL(k_lower_f32_to_f64, dim3(bx, m), dim3(256), 0, st, m, L32, ld32, L64, ld64);
}

}  // namespace pdas
