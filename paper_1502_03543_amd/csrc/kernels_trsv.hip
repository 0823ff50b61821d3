// The two triangular solves of the Cholesky route to dy (Section 5.1):
// L z = rhs, then L^T dy = z, with L row-major lower (ld).
//
// One kernel per solve, one workgroup per 64-row block.  Blocks are handed
// out by an atomic ticket in launch order, and a block waits (acquire) only
// on the ready flags of blocks with smaller tickets, which have all started,
// so the wait graph is acyclic.  Every wait is bounded: after ~2^22 polls the
// solve records an error in the iteration info and every block finishes.
//
// Off-diagonal blocks are applied as their flags are set; each block's
// coefficients are loaded before its flag is awaited, so only the short
// product with the newly published values sits on the critical path.  The
// 64 x 64 diagonal block is solved by one wavefront with its row (column) of
// L in registers and the solved entries broadcast with readlane (uniform
// operands, no memory traffic inside the recurrence).
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

constexpr int TB = kTB;
constexpr int kSpinLimit = 1 << 22;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Thread 0 waits until flag != 0; returns false when the solve is aborted.
__device__ bool wait_flag(int* flag, DevInfo* info, int* s_abort) {
  if (threadIdx.x == 0) {
    int spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      if (++spins > kSpinLimit ||
          __hip_atomic_load(&info->trsv_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        atomicOr(&info->trsv_err, 1);
        *s_abort = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  if (*s_abort) return false;
  // each thread acquires, so its later loads see the producer's stores
  (void)__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

__device__ inline void publish(int* flag) {
  __threadfence();
  __hip_atomic_store(flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_trsv_fwd(int m, const double* __restrict__ L, long ld,
                                                  const double* __restrict__ r, double* z,
                                                  int* sync, DevInfo* info) {
  __shared__ int s_rb, s_abort;
  __shared__ double Ld[TB][TB + 1];
  __shared__ double sacc[TB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) {
    s_rb = atomicAdd(&sync[0], 1);
    s_abort = 0;
  }
  __syncthreads();
  const int rb = s_rb;
  int* flags = sync + 4;
  const int i0 = rb * TB;
  const int rows = min(TB, m - i0);

  for (int e = tid; e < TB * TB; e += 256) {
    const int ii = e / TB, k = e % TB;
    double v = 0.0;
    if (ii < rows && k <= ii) v = L[(long)(i0 + ii) * ld + i0 + k];
    else if (ii == k) v = 1.0;
    Ld[ii][k] = v;
  }

  // off-diagonal blocks: wave wv owns rows wv, wv+4, ...; lane = column
  double acc[TB / 4];
#pragma unroll
  for (int k = 0; k < TB / 4; ++k) acc[k] = 0.0;
  for (int qb = 0; qb < rb; ++qb) {
    const int col = qb * TB + lane;
    double lv[TB / 4];
#pragma unroll
    for (int k = 0; k < TB / 4; ++k) {
      const int ii = wv + 4 * k;
      lv[k] = (ii < rows) ? L[(long)(i0 + ii) * ld + col] : 0.0;
    }
    if (!wait_flag(&flags[qb], info, &s_abort)) break;
    const double zc = z[col];
#pragma unroll
    for (int k = 0; k < TB / 4; ++k) acc[k] += lv[k] * zc;
  }
#pragma unroll
  for (int k = 0; k < TB / 4; ++k) {
    const double sv = wave_sum(acc[k]);
    if (lane == 0) sacc[wv + 4 * k] = sv;
  }
  __syncthreads();

  if (wv == 0) {
    double Lr[TB];
#pragma unroll
    for (int j = 0; j < TB; ++j) Lr[j] = Ld[lane][j];
    const double dl = 1.0 / Ld[lane][lane];
    double val = (lane < rows) ? (r[i0 + lane] - sacc[lane]) : 0.0;
    double mine = 0.0;
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      const double zj = readlane_d(val, j) * readlane_d(dl, j);
      if (lane == j) mine = zj;
      if (lane > j) val -= Lr[j] * zj;
    }
    if (lane < rows) z[i0 + lane] = mine;
    if (lane == 0) publish(&flags[rb]);
  }
}

__global__ __launch_bounds__(256) void k_trsv_bwd(int m, const double* __restrict__ L, long ld,
                                                  const double* __restrict__ zin, double* y,
                                                  int* sync, DevInfo* info) {
  __shared__ int s_rb, s_abort;
  __shared__ double Ld[TB][TB + 1];
  __shared__ double sacc[4][TB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nblk = (m + TB - 1) / TB;
  if (tid == 0) {
    s_rb = nblk - 1 - atomicAdd(&sync[1], 1);
    s_abort = 0;
  }
  __syncthreads();
  const int rb = s_rb;
  int* flags = sync + 4 + nblk;
  const int c0 = rb * TB;
  const int cols = min(TB, m - c0);

  for (int e = tid; e < TB * TB; e += 256) {
    const int ii = e / TB, k = e % TB;
    double v = 0.0;
    if (ii < cols && k <= ii) v = L[(long)(c0 + ii) * ld + c0 + k];
    else if (ii == k) v = 1.0;
    Ld[ii][k] = v;
  }

  // acc_c = sum over later blocks qb of sum_i L[i][c0 + c] y[i]; lane = column c
  double acc = 0.0;
  for (int qb = nblk - 1; qb > rb; --qb) {
    const int rows = min(TB, m - qb * TB);
    double lv[TB / 4];
#pragma unroll
    for (int k = 0; k < TB / 4; ++k) {
      const int ii = wv + 4 * k;
      lv[k] = (lane < cols && ii < rows) ? L[(long)(qb * TB + ii) * ld + c0 + lane] : 0.0;
    }
    if (!wait_flag(&flags[qb], info, &s_abort)) break;
#pragma unroll
    for (int k = 0; k < TB / 4; ++k) {
      const int ii = wv + 4 * k;
      if (ii < rows) acc += lv[k] * y[qb * TB + ii];
    }
  }
  sacc[wv][lane] = acc;
  __syncthreads();

  if (wv == 0) {
    // column `lane` of the diagonal block: Lc[j] = L[c0 + j][c0 + lane]
    double Lc[TB];
#pragma unroll
    for (int j = 0; j < TB; ++j) Lc[j] = Ld[j][lane];
    const double dl = 1.0 / Ld[lane][lane];
    const double tot = ((sacc[0][lane] + sacc[1][lane]) + sacc[2][lane]) + sacc[3][lane];
    double val = (lane < cols) ? (zin[c0 + lane] - tot) : 0.0;
    double mine = 0.0;
#pragma unroll
    for (int j = TB - 1; j >= 0; --j) {
      const double yj = readlane_d(val, j) * readlane_d(dl, j);
      if (lane == j) mine = yj;
      if (lane < j) val -= Lc[j] * yj;
    }
    if (lane < cols) y[c0 + lane] = mine;
    if (lane == 0) publish(&flags[rb]);
  }
}

}  // namespace

void launch_trsv_fwd(hipStream_t st, int m, const double* L, long ld, const double* r, double* z,
                     int* sync, DevInfo* info) {
  hipLaunchKernelGGL(k_trsv_fwd, dim3(cdiv(m, TB)), dim3(256), 0, st, m, L, ld, r, z, sync, info);
}

void launch_trsv_bwd(hipStream_t st, int m, const double* L, long ld, const double* z, double* y,
                     int* sync, DevInfo* info) {
  hipLaunchKernelGGL(k_trsv_bwd, dim3(cdiv(m, TB)), dim3(256), 0, st, m, L, ld, z, y, sync, info);
}

}  // namespace pdas
