// CPU emulation of the subset of HIP that the library's kernels use, for
// checking kernel logic on the host (test infrastructure only).
//
// Workgroups run one at a time, or (EMU_INTERLEAVE=K in the environment) K
// at a time on K OS threads, each taking the next workgroup in launch order;
// the threads of a workgroup are fibers on one OS thread
// (tests/emu/emu_runtime.cpp), and everything a workgroup owns (its thread
// and block indices, barriers, LDS) is thread-local, so concurrent
// workgroups interleave at arbitrary points and meet only in memory and in
// the (real) atomics.  A fiber runs until it waits at a
// barrier, so __syncthreads, wavefront exchanges (__shfl, __shfl_xor,
// readlane) and the matrix-core instructions (every lane of the wavefront
// contributes its operands, then each lane reads its result) follow the
// hardware's lock-step semantics, and a barrier that not every thread
// reaches is reported as a deadlock instead of hanging.  __shared__ becomes
// static storage (one workgroup at a time).  Memory is host memory, so
// AddressSanitizer sees every out-of-bounds access of a kernel.
#pragma once
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __shared__ static thread_local
#define __launch_bounds__(...)
#define HIP_SYMBOL(x) x

struct double2 { double x, y; };
struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph_t* hipGraph_t;
typedef struct ihipGraphExec_t* hipGraphExec_t;
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorUnknown = 999 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum { hipStreamCaptureModeThreadLocal = 0 };
enum { hipDeviceAttributeMultiprocessorCount = 0 };

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern thread_local dim3 threadIdx;
extern thread_local dim3 blockIdx, blockDim, gridDim;

// fiber scheduler (one OS thread): a fiber runs until it waits at a barrier
void emu_yield();
struct EmuBarrier {
  int count = 0, target = 0;
  long gen = 0;
  const char* name = "";
  // workgroup barriers: the source line the first thread of the current
  // generation waited at; every other thread must wait at the same line
  // (on the hardware a wavefront whose lanes reach two different barrier
  // instructions executes both, and the workgroup's count goes wrong)
  const char* site_file = nullptr;
  int site_line = 0;
  void init(int n, const char* nm) { target = n; count = 0; name = nm; site_file = nullptr; }
  void wait();
  void wait_at(const char* file, int line);
};
extern thread_local EmuBarrier g_block_bar;
constexpr int kEmuWaves = 16;  // up to 1024 threads per workgroup
extern thread_local EmuBarrier g_wave_bar[kEmuWaves];
extern thread_local uint64_t g_wave_buf[kEmuWaves][64];
extern thread_local uint64_t g_wave_buf2[kEmuWaves][64];
extern thread_local long g_barrier_count;
extern thread_local long g_progress;

inline void EmuBarrier::wait() {
  const long g = gen;
  if (++count == target) {
    count = 0;
    ++gen;
    ++g_progress;
    return;
  }
  while (gen == g) emu_yield();
}

inline void EmuBarrier::wait_at(const char* file, int line) {
  if (count == 0) {
    site_file = file;
    site_line = line;
  } else if (line != site_line || std::strcmp(file, site_file) != 0) {
    fprintf(stderr, "EMU BARRIER SITE MISMATCH block %u thread %u: %s:%d while the generation "
            "waits at %s:%d\n", blockIdx.x, threadIdx.x, file, line, site_file, site_line);
    std::abort();
  }
  wait();
}
inline void emu_syncthreads(const char* file, int line) {
  if (threadIdx.x == 0) ++g_barrier_count;
  g_block_bar.wait_at(file, line);
}
#define __syncthreads() emu_syncthreads(__FILE__, __LINE__)
inline void __threadfence() {}
// a wavefront runs in lock-step on the hardware; the emulation makes the
// points the kernels mark explicit synchronisation points of the wavefront
inline void __builtin_amdgcn_wave_barrier() { g_wave_bar[threadIdx.x >> 6].wait(); }
inline void __builtin_amdgcn_sched_barrier(int) {}
// instruction-scheduling hints: nothing to do on the host
inline void __builtin_amdgcn_iglp_opt(int) {}
inline void __builtin_amdgcn_s_setprio(int) {}
// with workgroups running at once, a polling thread gives its OS thread
// away for a moment (the producer it waits for runs on another one), so a
// spin limit counts real time as on the hardware rather than host loop trips
void emu_sleep();
inline void __builtin_amdgcn_s_sleep(int) { emu_sleep(); }
inline void __builtin_amdgcn_s_waitcnt(int) {}

template <typename T>
inline uint64_t emu_bits(T v) {
  uint64_t u = 0;
  std::memcpy(&u, &v, sizeof(T));
  return u;
}
template <typename T>
inline T emu_from(uint64_t u) {
  T v;
  std::memcpy(&v, &u, sizeof(T));
  return v;
}
template <typename T>
inline T emu_exchange(T v, int src) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  g_wave_buf[w][l] = emu_bits(v);
  g_wave_bar[w].wait();
  const T r = emu_from<T>(g_wave_buf[w][src & 63]);
  g_wave_bar[w].wait();
  return r;
}
template <typename T>
inline T __shfl_xor(T v, int o, int width = 64) {
  return emu_exchange(v, (threadIdx.x & 63) ^ o);
}
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  const int base = (threadIdx.x & 63) & ~(width - 1);
  return emu_exchange(v, base + (src & (width - 1)));
}
inline int __builtin_amdgcn_readlane(int v, int lane) { return emu_exchange(v, lane); }
// wavefront vote: nonzero when the predicate holds in any lane
inline int __any(int p) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  g_wave_buf[w][l] = p != 0;
  g_wave_bar[w].wait();
  int r = 0;
  for (int i = 0; i < 64; ++i) r |= g_wave_buf[w][i] != 0;
  g_wave_bar[w].wait();
  return r;
}

inline double __builtin_amdgcn_mfma_f64_4x4x4f64(double a, double b, double c, int, int, int) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  g_wave_buf[w][l] = emu_bits(a);
  g_wave_buf2[w][l] = emu_bits(b);
  g_wave_bar[w].wait();
  const int x = l & 3, blk = (l >> 2) & 3, y = l >> 4;
  double acc = c;
  for (int k = 0; k < 4; ++k) {
    const double av = emu_from<double>(g_wave_buf[w][y + 4 * blk + 16 * k]);
    const double bv = emu_from<double>(g_wave_buf2[w][x + 4 * blk + 16 * k]);
    acc = std::fma(av, bv, acc);
  }
  g_wave_bar[w].wait();
  return acc;
}

typedef double emu_d4 __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4f64: lane l holds A[i = l % 16][k = l / 16],
// B[k = l / 16][j = l % 16]; result slot v of lane l is D[l / 16 + 4 v][l % 16].
inline emu_d4 __builtin_amdgcn_mfma_f64_16x16x4f64(double a, double b, emu_d4 c, int, int, int) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  g_wave_buf[w][l] = emu_bits(a);
  g_wave_buf2[w][l] = emu_bits(b);
  g_wave_bar[w].wait();
  const int j = l % 16;
  emu_d4 r = c;
  for (int v = 0; v < 4; ++v) {
    const int i = l / 16 + 4 * v;
    double acc = r[v];
    for (int k = 0; k < 4; ++k)
      acc = std::fma(emu_from<double>(g_wave_buf[w][i + 16 * k]),
                     emu_from<double>(g_wave_buf2[w][j + 16 * k]), acc);
    r[v] = acc;
  }
  g_wave_bar[w].wait();
  return r;
}

inline double __builtin_amdgcn_rsq(double p) { return 1.0 / std::sqrt(p); }
inline float __builtin_amdgcn_rsqf(float p) { return 1.0f / std::sqrt(p); }
inline float __int_as_float(int v) { return emu_from<float>((uint32_t)v); }
inline int __float_as_int(float v) { return (int)(uint32_t)emu_bits(v); }
typedef float emu_f4 __attribute__((ext_vector_type(4)));
// v_mfma_f32_16x16x4f32: lane l holds A[i = l % 16][k = l / 16],
// B[j = l % 16][k = l / 16]; result lane l holds D[4 (l / 16) + v][l % 16].
inline emu_f4 __builtin_amdgcn_mfma_f32_16x16x4f32(float a, float b, emu_f4 c, int, int, int) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  g_wave_buf[w][l] = emu_bits(a);
  g_wave_buf2[w][l] = emu_bits(b);
  g_wave_bar[w].wait();
  const int j = l % 16;
  emu_f4 r = c;
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * (l / 16) + v;
    float acc = r[v];
    for (int k = 0; k < 4; ++k)
      acc = std::fma(emu_from<float>(g_wave_buf[w][i + 16 * k]), emu_from<float>(g_wave_buf2[w][j + 16 * k]), acc);
    r[v] = acc;
  }
  g_wave_bar[w].wait();
  return r;
}
// __hip_atomic_* are clang builtins in host code as well; their scope
// constants are predefined only in HIP mode
#ifndef __HIP_MEMORY_SCOPE_AGENT
#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#define __HIP_MEMORY_SCOPE_AGENT 4
#endif
inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline int atomicMin(int* p, int v) { return __atomic_fetch_min(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicMin(unsigned long long* p, unsigned long long v) {
  return __atomic_fetch_min(p, v, __ATOMIC_SEQ_CST);
}
inline int __double2loint(double d) { return (int)(uint32_t)emu_bits(d); }
inline int __double2hiint(double d) { return (int)(uint32_t)(emu_bits(d) >> 32); }
inline double __hiloint2double(int hi, int lo) { return emu_from<double>(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo); }
inline long long __double_as_longlong(double d) { return (long long)emu_bits(d); }
inline double __longlong_as_double(long long v) { return emu_from<double>((uint64_t)v); }
using std::isfinite;
using std::sqrt;
using std::min;
using std::max;

void emu_run_block(int nt, std::function<void()> body);
// dynamic LDS ("extern __shared__" arrays): a heap block of exactly the
// launch's size, refilled with NaN bytes before every workgroup (LDS holds
// no data from an earlier workgroup), so reads beyond it are reported and
// reads before a write show up as NaN
extern thread_local char* g_emu_dyn_lds;
int emu_interleave();  // workgroups run at once (EMU_INTERLEAVE, default 1)
// runs blocks first .. first + count - 1 (launch order, x fastest) of the
// grid on `workers` OS threads; each worker has its own LDS block
void emu_run_grid(dim3 grid, dim3 block, size_t shm, const std::function<void()>& body);
template <typename... KA, typename... A>
inline void emu_launch(void (*k)(KA...), dim3 grid, dim3 block, size_t shm, A... args) {
  emu_run_grid(grid, block, shm, [=] { k(args...); });
}
#define hipLaunchKernelGGL(k, grid, block, shm, st, ...) emu_launch(k, dim3(grid), dim3(block), (size_t)(shm), __VA_ARGS__)
enum { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
inline hipError_t hipFuncSetAttribute(const void*, int, int) { return hipSuccess; }

inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr) { return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, int, int) { *v = 4; return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, int) { return hipErrorUnknown; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { return hipErrorUnknown; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, void*, int) { return hipErrorUnknown; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorUnknown; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
