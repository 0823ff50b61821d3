// Sparse A (the first item of the paper's future work, Section 7: the same
// method for sparse systems, where keeping memory access coalesced is the
// difficulty).  A arrives as canonical CSR (column indices strictly
// increasing within a row); the library builds its transpose (CSC, row
// indices increasing within a column) once, so every product reads
// contiguous runs of indices and values:
//   A w        : G lanes per row of A (CSR),
//   A^T [v, u] : G lanes per column of A (CSC), both products at once,
// with G = 16 or 64 lanes chosen from the mean run length, and the normal
// matrix M = A D A^T (dense lower; the Cholesky stays dense): one wavefront
// forms row i as the sum over the entries a_ik of row i of (d_k a_ik) times
// the part of column k with rows j <= i, accumulated in an LDS row of
// length i + 1.  The work is sum_i sum_{k in row i} |{j <= i : a_jk != 0}|
// multiply-adds, against m^2 n / 2 for the dense product.  Every sum runs in
// a fixed order (entries k in increasing order; lanes in index order, then
// a fixed shuffle tree), so results are reproducible run to run.
#include <climits>
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

template <int G>
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Structure and values: row_ptr[0] == 0, 0 <= row_ptr[i] <= row_ptr[i + 1]
// <= nnz, row_ptr[m] == nnz, column indices in [0, n) and strictly
// increasing within a row (no duplicates), values finite.  Column indices
// of a row are read only after its bounds have been checked.  flags bit 0:
// bad structure, bit 1: non-finite value.
__global__ __launch_bounds__(256) void k_sp_check(long m, long n, long nnz,
                                                  const int64_t* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const double* __restrict__ v, int* flags) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long stride = (long)gridDim.x * blockDim.x;
  int bad = 0, nf = 0;
  if (t == 0) bad |= (rp[0] != 0) | (rp[m] != nnz);
  for (long i = t; i < m; i += stride) {
    const int64_t a = rp[i], b = rp[i + 1];
    if (!(0 <= a && a <= b && b <= nnz)) {
      bad = 1;
      continue;
    }
    int prev = -1;
    for (int64_t k = a; k < b; ++k) {
      const int c = ci[k];
      bad |= (c <= prev) | ((long)c >= n);
      prev = c;
    }
  }
  for (long k = t; k < nnz; k += stride) nf |= !isfinite(v[k]);
  if (bad) atomicOr(flags, 1);
  if (nf) atomicOr(flags, 2);
}

// CSC build (on checked structure): counts per column, an exclusive scan,
// each row's entries placed with a per-column cursor, then each column put
// in row order (the cursor order depends on scheduling; the sort removes
// that), and the position of every CSR entry in the CSC recorded.
__global__ void k_sp_count(long nnz, const int* __restrict__ ci, int* cnt) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&cnt[ci[k]], 1);
}

// cp[0] = 0, cp[j + 1] = cp[j] + cnt[j] (one workgroup, chunks of 256 with
// a running total); cur[j] = cp[j].
__global__ __launch_bounds__(256) void k_sp_scan(long n, const int* __restrict__ cnt,
                                                 int64_t* cp, int* cur) {
  __shared__ int64_t part[256];
  __shared__ int64_t base;
  if (threadIdx.x == 0) {
    base = 0;
    cp[0] = 0;
  }
  __syncthreads();
  for (long j0 = 0; j0 < n; j0 += 256) {
    const long j = j0 + threadIdx.x;
    part[threadIdx.x] = j < n ? cnt[j] : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t run = base;
      for (int k = 0; k < 256; ++k) {
        run += part[k];
        part[k] = run;  // inclusive
      }
      base = run;
    }
    __syncthreads();
    if (j < n) {
      cp[j + 1] = part[threadIdx.x];
      cur[j] = (int)(part[threadIdx.x] - cnt[j]);
    }
    __syncthreads();
  }
}

__global__ void k_sp_fill(long m, const int64_t* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ v, int* cur, int* __restrict__ ri,
                          double* __restrict__ cv, int* __restrict__ src) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= m) return;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
    const int pos = atomicAdd(&cur[ci[k]], 1);
    ri[pos] = (int)i;
    cv[pos] = v[k];
    src[pos] = (int)k;
  }
}

__global__ void k_sp_sort(long n, const int64_t* __restrict__ cp, int* __restrict__ ri,
                          double* __restrict__ cv, int* __restrict__ src) {
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t a = cp[j], b = cp[j + 1];
  for (int64_t k = a + 1; k < b; ++k) {  // insertion sort by row (distinct rows)
    const int r = ri[k], s = src[k];
    const double x = cv[k];
    int64_t q = k - 1;
    while (q >= a && ri[q] > r) {
      ri[q + 1] = ri[q];
      cv[q + 1] = cv[q];
      src[q + 1] = src[q];
      --q;
    }
    ri[q + 1] = r;
    cv[q + 1] = x;
    src[q + 1] = s;
  }
}

__global__ void k_sp_map(long nnz, const int* __restrict__ src, int* __restrict__ map) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p < nnz) map[src[p]] = (int)p;
}

// out[i] = base[i] + sign * sum_k A_ik w_k: G lanes per row (CSR).
template <int G>
__global__ __launch_bounds__(256) void k_sp_gemv_n(long m, const int64_t* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ w,
                                                   const double* __restrict__ base, double sign,
                                                   double* out) {
  const long i = blockIdx.x * (256L / G) + (threadIdx.x / G);
  const int lane = threadIdx.x % G;
  const bool live = i < m;  // every lane stays for the shuffles
  double acc = 0.0;
  if (live)
    for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += G) acc += v[k] * w[ci[k]];
  acc = group_sum<G>(acc);
  if (live && lane == 0) out[i] = base[i] + sign * acc;
}

// g1[j] = sum_i A_ij v1_i and (when v2) g2[j] = sum_i A_ij v2_i: G lanes
// per column (CSC).
template <int G>
__global__ __launch_bounds__(256) void k_sp_gemv_t(long n, const int64_t* __restrict__ cp,
                                                   const int* __restrict__ ri,
                                                   const double* __restrict__ cv,
                                                   const double* __restrict__ v1,
                                                   const double* __restrict__ v2, double* g1,
                                                   double* g2) {
  const long j = blockIdx.x * (256L / G) + (threadIdx.x / G);
  const int lane = threadIdx.x % G;
  const bool live = j < n;
  double a1 = 0.0, a2 = 0.0;
  if (live)
    for (int64_t k = cp[j] + lane; k < cp[j + 1]; k += G) {
      const double a = cv[k];
      const int r = ri[k];
      a1 += a * v1[r];
      if (v2) a2 += a * v2[r];
    }
  a1 = group_sum<G>(a1);
  if (v2) a2 = group_sum<G>(a2);
  if (live && lane == 0) {
    g1[j] = a1;
    if (v2) g2[j] = a2;
  }
}

// Row i of M (j <= i), one wavefront per row, rows taken largest first.
// The entries e = (i, k) of row i are read 64 at a time, lane t holding
// entry t's scale u = d_k a_ik and the run of column k with rows <= i (it
// ends at (i, k) itself, whose CSC position map[e] gives); then entry after
// entry, in increasing k, the lanes add u a_jk into the LDS row accumulator
// over the run (rows j distinct within a run, so lanes never collide).  A
// wavefront's LDS accesses take effect in program order, so the entries
// need no barrier between them, and the next entry's run is loaded while
// the current one is added.
__global__ __launch_bounds__(64) void k_sp_syrk(long m, const int64_t* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const double* __restrict__ v,
                                                const int64_t* __restrict__ cp,
                                                const int* __restrict__ ri,
                                                const double* __restrict__ cv,
                                                const int* __restrict__ map,
                                                const double* __restrict__ d, double* M,
                                                long ldm) {
  extern __shared__ double lds[];
  double* acc = lds;  // m (i + 1 used)
  const long i = m - 1 - blockIdx.x;
  const int lane = threadIdx.x;
  for (long j = lane; j <= i; j += 64) acc[j] = 0.0;
  const int64_t e0 = rp[i], e1 = rp[i + 1];
  for (int64_t eb = e0; eb < e1; eb += 64) {
    const int ne = (int)min((int64_t)64, e1 - eb);
    double u_l = 0.0;
    long p0_l = 0;
    int len_l = 0;
    if (lane < ne) {
      const int64_t e = eb + lane;
      const int k = ci[e];
      p0_l = (long)cp[k];
      u_l = d[k] * v[e];
      len_l = (int)(map[e] - p0_l + 1);
    }
    // entry 0 of the chunk: its run's first 64 entries
    long p0 = __shfl(p0_l, 0, 64);
    int len = __shfl(len_l, 0, 64);
    int rj = lane < len ? ri[p0 + lane] : 0;
    double rv = lane < len ? cv[p0 + lane] : 0.0;
    for (int q = 0; q < ne; ++q) {
      const double u = __shfl(u_l, q, 64);
      const long p0c = p0;
      const int lenc = len;
      const int rjc = rj;
      const double rvc = rv;
      // the next entry's run, in flight while this one is added
      if (q + 1 < ne) {
        p0 = __shfl(p0_l, q + 1, 64);
        len = __shfl(len_l, q + 1, 64);
        rj = lane < len ? ri[p0 + lane] : 0;
        rv = lane < len ? cv[p0 + lane] : 0.0;
      }
      if (lane < lenc) acc[rjc] += u * rvc;
      for (int t = 64 + lane; t < lenc; t += 64) acc[ri[p0c + t]] += u * cv[p0c + t];
    }
  }
  // every lane's last additions precede the reads below (in issue order on
  // the hardware; marked so for the compiler and the host emulation)
  __builtin_amdgcn_wave_barrier();
  double* Mi = M + i * ldm;
  for (long j = lane; j <= i; j += 64) Mi[j] = acc[j];
}

inline bool wide_runs(long nnz, long runs) { return runs > 0 && nnz >= 48 * runs; }

}  // namespace

size_t sp_syrk_lds_bytes(long m) { return (size_t)m * sizeof(double); }

bool sp_fits(long m) { return sp_syrk_lds_bytes(m) <= kSparseMaxLds; }

hipError_t sp_prepare() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_sp_syrk),
                             hipFuncAttributeMaxDynamicSharedMemorySize, kSparseMaxLds);
}

void launch_sp_check(hipStream_t st, long m, long n, long nnz, const int64_t* rp, const int* ci,
                     const double* v, int* flags) {
  const long work = nnz > m ? nnz : m;
  int blocks = cdiv(work, 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_sp_check, dim3(blocks), dim3(256), 0, st, m, n, nnz, rp, ci, v, flags);
}

void launch_sp_transpose(hipStream_t st, long m, long n, long nnz, const int64_t* rp,
                         const int* ci, const double* v, int* cnt, int* cur, int64_t* cp,
                         int* ri, double* cv, int* src, int* map) {
  launch_fill_i32(st, cnt, 0, n);
  if (nnz > 0)
    hipLaunchKernelGGL(k_sp_count, dim3(cdiv(nnz, 256)), dim3(256), 0, st, nnz, ci, cnt);
  hipLaunchKernelGGL(k_sp_scan, dim3(1), dim3(256), 0, st, n, cnt, cp, cur);
  hipLaunchKernelGGL(k_sp_fill, dim3(cdiv(m, 256)), dim3(256), 0, st, m, rp, ci, v, cur, ri, cv,
                     src);
  hipLaunchKernelGGL(k_sp_sort, dim3(cdiv(n, 256)), dim3(256), 0, st, n, cp, ri, cv, src);
  if (nnz > 0) hipLaunchKernelGGL(k_sp_map, dim3(cdiv(nnz, 256)), dim3(256), 0, st, nnz, src, map);
}

void launch_sp_gemv_n(hipStream_t st, long m, long nnz, const int64_t* rp, const int* ci,
                      const double* v, const double* w, const double* base, double* out,
                      double sign) {
  if (wide_runs(nnz, m))
    hipLaunchKernelGGL(k_sp_gemv_n<64>, dim3(cdiv(m, 4)), dim3(256), 0, st, m, rp, ci, v, w, base,
                       sign, out);
  else
    hipLaunchKernelGGL(k_sp_gemv_n<16>, dim3(cdiv(m, 16)), dim3(256), 0, st, m, rp, ci, v, w,
                       base, sign, out);
}

void launch_sp_gemv_t(hipStream_t st, long n, long nnz, const int64_t* cp, const int* ri,
                      const double* cv, const double* v1, const double* v2, double* g1,
                      double* g2) {
  if (wide_runs(nnz, n))
    hipLaunchKernelGGL(k_sp_gemv_t<64>, dim3(cdiv(n, 4)), dim3(256), 0, st, n, cp, ri, cv, v1, v2,
                       g1, g2);
  else
    hipLaunchKernelGGL(k_sp_gemv_t<16>, dim3(cdiv(n, 16)), dim3(256), 0, st, n, cp, ri, cv, v1,
                       v2, g1, g2);
}

void launch_sp_syrk(hipStream_t st, long m, const int64_t* rp, const int* ci, const double* v,
                    const int64_t* cp, const int* ri, const double* cv, const int* map,
                    const double* d, double* M, long ldm) {
  hipLaunchKernelGGL(k_sp_syrk, dim3(m), dim3(64), sp_syrk_lds_bytes(m), st, m, rp, ci, v, cp,
                     ri, cv, map, d, M, ldm);
}

}  // namespace pdas
