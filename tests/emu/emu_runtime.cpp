// Fiber scheduler of the HIP emulation (x86-64 System V): each thread of a
// workgroup is a fiber with its own stack; emu_switch saves the callee-saved
// registers and swaps stacks.
#include "hip/hip_runtime.h"
#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/asan_interface.h>
#define EMU_UNPOISON(p, n) __asan_unpoison_memory_region(p, n)
#else
#define EMU_UNPOISON(p, n) ((void)0)
#endif

#include <atomic>
#include <thread>

thread_local dim3 threadIdx;
thread_local dim3 blockIdx, blockDim, gridDim;
thread_local EmuBarrier g_block_bar;
thread_local EmuBarrier g_wave_bar[kEmuWaves];
thread_local uint64_t g_wave_buf[kEmuWaves][64];
thread_local uint64_t g_wave_buf2[kEmuWaves][64];
thread_local long g_barrier_count = 0;
thread_local char* g_emu_dyn_lds = nullptr;
thread_local long g_progress = 0;

extern "C" void emu_switch(void** save_sp, void* load_sp);
asm(R"(
.text
.globl emu_switch
.type emu_switch,@function
emu_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
)");

namespace {
constexpr size_t kStack = 256 * 1024;
struct Fiber { void* sp = nullptr; bool done = false; };
thread_local void* g_main_sp = nullptr;
thread_local std::vector<Fiber> g_f;
thread_local std::vector<char> g_stacks;
thread_local std::function<void()> g_body;
thread_local int g_cur = -1;
extern "C" void emu_entry() {
  const int t = g_cur;
  threadIdx = dim3(t, 0, 0);
  g_body();
  g_f[t].done = true;
  ++g_progress;
  emu_switch(&g_f[t].sp, g_main_sp);
  std::abort();
}
}  // namespace

void emu_yield() {
  const int t = g_cur;
  emu_switch(&g_f[t].sp, g_main_sp);
  threadIdx = dim3(t, 0, 0);
}

void emu_run_block(int nt, std::function<void()> body) {
  g_body = std::move(body);
  g_block_bar.init(nt, "block");
  if (nt > 64 * kEmuWaves) {
    fprintf(stderr, "EMU: %d threads per workgroup exceed %d\n", nt, 64 * kEmuWaves);
    std::abort();
  }
  for (int w = 0; w < kEmuWaves; ++w) g_wave_bar[w].init(64, "wave");
  g_f.assign(nt, Fiber{});
  if (g_stacks.size() < (size_t)nt * kStack) g_stacks.resize((size_t)nt * kStack);
  EMU_UNPOISON(g_stacks.data(), g_stacks.size());
  for (int t = 0; t < nt; ++t) {
    uintptr_t top = (uintptr_t)(g_stacks.data() + (size_t)(t + 1) * kStack);
    top &= ~(uintptr_t)15;
    void** sp = (void**)top;
    *--sp = nullptr;                     // fake return address of emu_entry
    *--sp = (void*)&emu_entry;           // ret target
    for (int r = 0; r < 6; ++r) *--sp = nullptr;
    g_f[t].sp = sp;
  }
  int stuck = 0;
  for (;;) {
    const long before = g_progress;
    bool any = false;
    for (int t = 0; t < nt; ++t) {
      if (g_f[t].done) continue;
      any = true;
      g_cur = t;
      emu_switch(&g_main_sp, g_f[t].sp);
    }
    if (!any) break;
    if (g_progress == before) {
      if (++stuck > 3) {
        int alive = 0;
        for (auto& f : g_f) alive += !f.done;
        fprintf(stderr, "EMU DEADLOCK block %u: %d threads alive, block barrier %d/%d arrived,"
                " wave barriers %d %d %d %d\n", blockIdx.x, alive, g_block_bar.count,
                g_block_bar.target, g_wave_bar[0].count, g_wave_bar[1].count,
                g_wave_bar[2].count, g_wave_bar[3].count);
        std::abort();
      }
    } else {
      stuck = 0;
    }
  }
}

int emu_interleave() {
  static const int k = [] {
    const char* e = std::getenv("EMU_INTERLEAVE");
    const int v = e ? std::atoi(e) : 1;
    return v < 1 ? 1 : (v > 64 ? 64 : v);
  }();
  return k;
}

void emu_run_grid(dim3 grid, dim3 block, size_t shm, const std::function<void()>& body) {
  const long nblocks = (long)grid.x * grid.y;
  const int workers = (int)std::min<long>(emu_interleave(), nblocks);
  std::atomic<long> next{0};
  auto work = [&] {
    blockDim = block;
    gridDim = grid;
    char* dyn = shm ? new char[shm] : nullptr;
    g_emu_dyn_lds = dyn;
    for (long b = next.fetch_add(1); b < nblocks; b = next.fetch_add(1)) {
      blockIdx = dim3((unsigned)(b % grid.x), (unsigned)(b / grid.x), 0);
      if (dyn) std::memset(dyn, 0xff, shm);
      emu_run_block(block.x, body);
    }
    delete[] dyn;
    g_emu_dyn_lds = nullptr;
  };
  if (workers <= 1) {
    work();
    return;
  }
  std::vector<std::thread> pool;
  for (int w = 0; w < workers; ++w) pool.emplace_back(work);
  for (auto& t : pool) t.join();
}

void emu_sleep() {
  if (emu_interleave() > 1) std::this_thread::sleep_for(std::chrono::microseconds(20));
}
