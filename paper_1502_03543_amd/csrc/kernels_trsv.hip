// The two triangular solves of the Cholesky route to dy (Section 5.1):
// L z = rhs, then L^T dy = z, with L row-major lower (ld).
//
// One kernel per solve, one workgroup per 64-row block.  Blocks are handed
// out by an atomic ticket in launch order, and a block waits only on blocks
// with smaller tickets, which have all started, so the wait graph is
// acyclic.  Every wait is bounded: after ~2^22 polls the solve records an
// error in the iteration info and every block finishes.  Each block loads
// the coefficients of a block below (above) before waiting for it, so only
// the short product with the newly solved values sits on the critical path.
//
// Forward solve: a ready flag per block (release / acquire); the 64 x 64
// diagonal block is solved by one wavefront with its row of L in registers
// and the solved entries broadcast with readlane.
// Backward solve (every iteration): the solution entries themselves are the
// ready signal (see k_trsv_bwd), and the diagonal block is solved in four
// 16 x 16 steps with the inverses of its diagonal sub-blocks, which each
// workgroup forms while the blocks below it are being solved.
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

// Thread 0 waits until flag != 0 (relaxed polls; the acquire follows once,
// in every thread); returns false when the solve is aborted.
__device__ bool wait_flag(int* flag, DevInfo* info, int* s_abort) {
  if (threadIdx.x == 0) {
    int spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
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
  const bool abort = *s_abort != 0;
  // every thread has the verdict before thread 0, running ahead into the
  // next wait, can set the flag on a timeout (the others would then leave
  // the loop one wait early and meet a different barrier)
  __syncthreads();
  if (abort) return false;
  // each thread acquires, so its later loads see the producer's stores
  (void)__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// The release store orders this wavefront's earlier stores (the solved
// entries) before the flag.
__device__ inline void publish(int* flag) {
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

// Backward solve L^T y = z.  A block's solution entries are its own ready
// signal: y holds kPending (a NaN payload no arithmetic produces) before the
// launch, every entry is written once with a device-coherent store, and a
// reader polls the entries it needs until none is pending.  No flag and no
// cache flush sit between a block's result and the blocks above it.
constexpr unsigned long long kPending = 0x7ff4dead0000beefull;
constexpr int SB = 16;  // sub-block of the diagonal solve

__device__ inline bool pending(double v) {
  return (unsigned long long)__double_as_longlong(v) == kPending;
}

__global__ __launch_bounds__(256) void k_fill_pending(double* y, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) y[i] = __longlong_as_double((long long)kPending);
}

__global__ __launch_bounds__(256) void k_trsv_bwd(int m, const double* __restrict__ L, long ld,
                                                  const double* __restrict__ zin, double* y,
                                                  int* sync, DevInfo* info) {
  __shared__ int s_rb;
  __shared__ double Ld[TB][TB + 1];
  __shared__ double Xi[TB / SB][SB][SB + 1];  // inverses of the 16 x 16 diagonal sub-blocks
  __shared__ double sacc[4][TB];
  __shared__ double tb[TB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nblk = (m + TB - 1) / TB;
  if (tid == 0) s_rb = nblk - 1 - atomicAdd(&sync[1], 1);
  __syncthreads();
  const int rb = s_rb;
  const int c0 = rb * TB;
  const int cols = min(TB, m - c0);

  for (int e = tid; e < TB * TB; e += 256) {
    const int ii = e / TB, k = e % TB;
    double v = 0.0;
    if (ii < cols && k <= ii) v = L[(long)(c0 + ii) * ld + c0 + k];
    else if (ii == k) v = 1.0;
    Ld[ii][k] = v;
  }
  __syncthreads();

  // wavefront w inverts diagonal sub-block w, lane l < 16 forming column l
  // of its inverse by forward substitution (done while the blocks below are
  // still being solved, so off the critical path except for the last block)
  if (lane < SB) {
    const int o = SB * wv;
    double x[SB], rd[SB];
#pragma unroll
    for (int i = 0; i < SB; ++i) rd[i] = 1.0 / Ld[o + i][o + i];
#pragma unroll
    for (int i = 0; i < SB; ++i) {
      double v = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) v = fma(-Ld[o + i][o + k], x[k], v);
      x[i] = v * rd[i];
      Xi[wv][i][lane] = x[i];
    }
  }

  // the diagonal step's operands, loaded before the waits: column `lane` of
  // the diagonal block, column lane % 16 of its sub-block's inverse, z
  __syncthreads();
  double Lc[TB], xc[SB];
  const int sl = lane / SB, ll = lane % SB;
  const double zc = (lane < cols) ? zin[c0 + lane] : 0.0;
  if (wv == 0) {
#pragma unroll
    for (int j = 0; j < TB; ++j) Lc[j] = Ld[j][lane];
#pragma unroll
    for (int j = 0; j < SB; ++j) xc[j] = Xi[sl][j][ll];
  }

  // acc_c = sum over later blocks qb of sum_i L[i][c0 + c] y[i]; lane =
  // column c, wavefront w takes rows 16 w .. 16 w + 15 of each block: one
  // 128-byte line of y, which it polls with one coalesced load
  double acc = 0.0;
  bool abort = false;
  for (int qb = nblk - 1; qb > rb && !abort; --qb) {
    const int rows = min(TB, m - qb * TB);
    const int r0 = SB * wv, nr = min(SB, rows - r0);
    if (nr <= 0) continue;
    const double* yq = y + qb * TB + r0;
    double lv[SB], yv[SB];
#pragma unroll
    for (int k = 0; k < SB; ++k)
      lv[k] = (lane < cols && k < nr) ? L[(long)(qb * TB + r0 + k) * ld + c0 + lane] : 0.0;
    for (int spins = 0;; ++spins) {
      // lane k loads entry k % 16 of the line: one coalesced access per poll,
      // and once none is pending the values are already here
      const int k16 = min(lane & (SB - 1), nr - 1);
      const double v = __hip_atomic_load(&yq[k16], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!__any(pending(v))) {
#pragma unroll
        for (int k = 0; k < SB; ++k) yv[k] = (k < nr) ? readlane_d(v, k) : 0.0;
        break;
      }
      if (spins > kSpinLimit ||
          __hip_atomic_load(&info->trsv_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        if (lane == 0) atomicOr(&info->trsv_err, 1);
        abort = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int k = 0; k < SB; ++k) acc += lv[k] * yv[k];
  }
  sacc[wv][lane] = acc;
  __syncthreads();

  if (wv == 0) {
    // L_bb^T y = t in four steps from the last sub-block: y_s = X_s^T t_s,
    // then t_r -= L[s rows][r cols]^T y_s for the sub-blocks r < s
    const double tot = ((sacc[0][lane] + sacc[1][lane]) + sacc[2][lane]) + sacc[3][lane];
    double t = (lane < cols) ? (zc - tot) : 0.0;
    double mine = 0.0;
#pragma unroll
    for (int s = TB / SB - 1; s >= 0; --s) {
      tb[lane] = t;
      __builtin_amdgcn_wave_barrier();
      double ys = 0.0;
#pragma unroll
      for (int j = 0; j < SB; ++j) ys = fma(xc[j], tb[SB * s + j], ys);
      if (sl == s) mine = ys;
      if (s == 0) break;
      __builtin_amdgcn_wave_barrier();
      tb[lane] = ys;
      __builtin_amdgcn_wave_barrier();
      if (sl < s) {
#pragma unroll
        for (int j = 0; j < SB; ++j) t = fma(-Lc[SB * s + j], tb[SB * s + j], t);
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (lane < cols)
      __hip_atomic_store(&y[c0 + lane], mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

void launch_trsv_fwd(hipStream_t st, int m, const double* L, long ld, const double* r, double* z,
                     int* sync, DevInfo* info) {
  hipLaunchKernelGGL(k_trsv_fwd, dim3(cdiv(m, TB)), dim3(256), 0, st, m, L, ld, r, z, sync, info);
}

void launch_trsv_bwd(hipStream_t st, int m, const double* L, long ld, const double* z, double* y,
                     int* sync, DevInfo* info) {
  hipLaunchKernelGGL(k_fill_pending, dim3(cdiv(m, 256)), dim3(256), 0, st, y, m);
  hipLaunchKernelGGL(k_trsv_bwd, dim3(cdiv(m, TB)), dim3(256), 0, st, m, L, ld, z, y, sync, info);
}

}  // namespace pdas
