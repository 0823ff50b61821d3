// Allocation-free variant of lp_chol_solve for callers that cannot allocate
// device memory or pass a workspace (code under stream capture, tight
// serving loops): its scratch (the iteration record, the triangular solves'
// tickets and flags, and the intermediate z = L^-1 r) lives in one
// file-scope device array per GPU.
//
// In host code the name `scratch` stands for the host-side shadow of that
// array, not a device address.  Its device address is taken once per device
// with hipGetSymbolAddress, with that device current, and only that address
// is ever handed to kernels.
#include <climits>
#include <mutex>

#include "pdas_internal.h"

using namespace pdas;

namespace {

constexpr int kNoAllocMaxM = LP_NOALLOC_MAX_M;
static_assert(kNoAllocMaxM % kTB == 0, "whole triangular-solve blocks");
constexpr size_t kAlign = 256;

constexpr size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
// layout: DevInfo | sync ints (4 + 2 * blocks) | z (m doubles)
constexpr size_t kInfoOff = 0;
constexpr size_t kSyncOff = align_up(sizeof(DevInfo));
constexpr size_t kSyncInts = 4 + 2 * ((kNoAllocMaxM + kTB - 1) / kTB);
constexpr size_t kZOff = align_up(kSyncOff + kSyncInts * sizeof(int));
constexpr size_t kScratchBytes = align_up(kZOff + (size_t)kNoAllocMaxM * sizeof(double));

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on each device).  nullptr on failure.
unsigned char* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[dev] = p;
  }
  return static_cast<unsigned char*>(g_ptr[dev]);
}

}  // namespace

extern "C" {

lp_status lp_chol_solve_noalloc(int64_t m, const double* L, int64_t ldm, const double* r,
                                double* dy, lp_stream_t stream) {
  if (!L || !r || !dy || r == dy || ldm < m) return LP_ERR_INVALID_ARG;
  if (m < 1) return LP_ERR_SHAPE;
  if (m > kNoAllocMaxM) return LP_ERR_WORKSPACE;
  unsigned char* base = scratch_on_current_device();
  if (!base) return LP_ERR_DEVICE;
  DevInfo* info = reinterpret_cast<DevInfo*>(base + kInfoOff);
  int* sync = reinterpret_cast<int*>(base + kSyncOff);
  double* z = reinterpret_cast<double*>(base + kZOff);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the tickets and flags must start at zero: cleared by a kernel (no memset
  // node, so the call can be captured)
  launch_iter_begin(s, info, sync, cdiv(m, kTB));
  launch_trsv_fwd(s, (int)m, L, ldm, r, z, sync, info);
  launch_trsv_bwd(s, (int)m, L, ldm, z, dy, sync, info);
  return hipGetLastError() == hipSuccess ? LP_OK : LP_ERR_DEVICE;
}

}  // extern "C"
