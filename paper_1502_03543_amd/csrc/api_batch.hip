// C ABI of the batched solver: many independent LPs, each advanced by the
// Section 3 iteration.  One iteration of the whole batch is a fixed sequence
// of launches (see kernels_batch.hip); several iterations are captured into
// one hipGraph and replayed until no LP remains active.  The library allocates no device memory: everything is
// carved from the caller's workspace.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "pdas_internal.h"

using namespace pdas;

namespace {

constexpr size_t kAlign = 256;
constexpr int kItersPerGraph = 4;  // default of lp_options.batch_graph_iters
constexpr int kCompactMin = 8;     // no compaction below this many launched LPs
constexpr int kMaxBatchRefine = 16;  // largest lp_options.refine_max of a mixed batch

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Gather the caller's vectors (arbitrary offsets) into the packed layout, and
// check finiteness / interior start per LP.
__global__ __launch_bounds__(256) void k_batch_gather(int count, const BatchLP* lps,
                                                      const long long* uvm,
                                                      const long long* uvn, const double* b,
                                                      const double* c, const double* x0,
                                                      const double* y0, const double* s0,
                                                      const double* A, double* pb, double* pc,
                                                      double* px, double* py, double* ps,
                                                      int* flags) {
  const int lp = blockIdx.x;
  if (lp >= count) return;
  const BatchLP P = lps[lp];
  int bad = 0, nonpos = 0;
  for (int i = threadIdx.x; i < P.m; i += 256) {
    const double bv = b[uvm[lp] + i], yv = y0[uvm[lp] + i];
    pb[P.vm + i] = bv;
    py[P.vm + i] = yv;
    bad |= !isfinite(bv) | !isfinite(yv);
  }
  for (int j = threadIdx.x; j < P.n; j += 256) {
    const double cv = c[uvn[lp] + j], xv = x0[uvn[lp] + j], sv = s0[uvn[lp] + j];
    pc[P.vn + j] = cv;
    px[P.vn + j] = xv;
    ps[P.vn + j] = sv;
    bad |= !isfinite(cv) | !isfinite(xv) | !isfinite(sv);
    nonpos |= !(xv > 0) | !(sv > 0);
  }
  const long mn = (long)P.m * P.n;
  for (long e = threadIdx.x; e < mn; e += 256) bad |= !isfinite(A[P.a_off + e]);
  if (bad) atomicOr(&flags[lp], 1);
  if (nonpos) atomicOr(&flags[lp], 2);
}

__global__ void k_batch_init_state(int count, BatchState* st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  BatchState s{};
  s.status = LP_OK;
  s.iters = 0;
  s.cur = 0;
  s.gap = 0.0;
  s.last_psi = 0.0;
  s.last_t = 0.0;
  s.last_argmax = -1;
  st[i] = s;
}

__global__ void k_batch_copy_cur(int count, const BatchLP* lps, const BatchState* st,
                                 double* const* xb, double* const* yb, double* const* sb,
                                 double* x, double* y, double* s) {
  const int lp = blockIdx.x;
  if (lp >= count) return;
  const BatchLP P = lps[lp];
  const int cur = st[lp].cur;
  for (int j = threadIdx.x; j < P.n; j += blockDim.x) {
    if (x) x[P.vn + j] = xb[cur][P.vn + j];
    if (s) s[P.vn + j] = sb[cur][P.vn + j];
  }
  for (int i = threadIdx.x; i < P.m; i += blockDim.x)
    if (y) y[P.vm + i] = yb[cur][P.vm + i];
}

__global__ void k_batch_tape_row(int count, const BatchLP* lps, const BatchState* st,
                                 const double* tape, int k, double* x, double* y, double* s) {
  const int lp = blockIdx.x;
  if (lp >= count || k >= st[lp].iters) return;
  const BatchLP P = lps[lp];
  const double* r = tape + P.tape_off + (long)k * (3 * P.n + P.m);
  for (int j = threadIdx.x; j < P.n; j += blockDim.x) {
    if (x) x[P.vn + j] = r[j];
    if (s) s[P.vn + j] = r[P.n + P.m + j];
  }
  for (int i = threadIdx.x; i < P.m; i += blockDim.x)
    if (y) y[P.vm + i] = r[P.n + i];
}

}  // namespace

struct lp_batch {
  int count = 0;
  int graph_iters = kItersPerGraph;
  lp_options opt{};
  hipStream_t st = nullptr;
  std::vector<BatchLP> lps_h;
  long sum_m = 0, sum_n = 0;
  BatchArgs args{};
  BatchLP* lps = nullptr;
  BatchState* state = nullptr;
  double* bufptrs = nullptr;  // device copies of the iterate buffer pointers
  int* flags = nullptr;
  long long* uvm = nullptr;   // caller's vector offsets (device copies)
  long long* uvn = nullptr;
  BatchAdj adj{};             // reverse-sweep pools (with a tape)
  int max_iters_run = 0;
  int max_m = 0;
  int max_tiles = 0;          // 64 x 64 tiles of the largest A (for Abar)
  std::vector<int> order;     // descriptor slot -> caller's LP index
};

namespace {

bool batch_shapes_ok(int32_t count, const int64_t* m, const int64_t* n) {
  if (count < 1 || !m || !n) return false;
  for (int i = 0; i < count; ++i)
    if (m[i] < 1 || n[i] <= m[i] || n[i] > INT_MAX / 4) return false;
  return true;
}

void carve_batch(lp_batch* h, const int64_t* m, const int64_t* n, Carver& cv) {
  const int count = h->count;
  h->lps_h.resize(count);
  long vm = 0, vn = 0, moff = 0, toff = 0, doff = 0, a32 = 0, m32 = 0, vn4 = 0;
  const int tape_cap = h->opt.tape_capacity > 0 ? h->opt.tape_capacity : 0;
  for (int i = 0; i < count; ++i) {
    BatchLP& P = h->lps_h[i];
    P.m = (int)m[i];
    P.n = (int)n[i];
    P.ldm = (P.m + 7) / 8 * 8;
    P.pad = 0;
    P.a_off = 0;
    P.vm = vm;
    P.vn = vn;
    P.M_off = moff;
    P.tape_off = toff;
    P.diag_off = doff;
    P.n4 = (P.n + 3) / 4 * 4;
    P.ld32 = (P.m + 3) / 4 * 4;
    P.a32_off = a32;
    P.m32_off = m32;
    P.vn4 = vn4;
    a32 += (long)P.m * P.n4;
    m32 += (long)P.ld32 * P.m;
    vn4 += P.n4;
    doff += potrf_diag_elems(P.m);
    vm += P.m;
    vn += P.n;
    moff += (long)P.ldm * P.m;
    toff += (long)(tape_cap + 1) * (3 * P.n + P.m);
  }
  h->sum_m = vm;
  h->sum_n = vn;
  BatchArgs& a = h->args;
  a.count = count;
  h->lps = cv.take<BatchLP>(count);
  h->state = cv.take<BatchState>(count);
  h->flags = cv.take<int>(count);
  h->uvm = cv.take<long long>(count);
  h->uvn = cv.take<long long>(count);
  a.b = cv.take<double>(vm);
  a.c = cv.take<double>(vn);
  for (int k = 0; k < 2; ++k) {
    a.x[k] = cv.take<double>(vn);
    a.y[k] = cv.take<double>(vm);
    a.s[k] = cv.take<double>(vn);
    a.rd[k] = cv.take<double>(vn);
  }
  a.d = cv.take<double>(vn);
  a.w = cv.take<double>(vn);
  a.g = cv.take<double>(vn);
  a.gy = cv.take<double>(vn);
  a.dx = cv.take<double>(vn);
  a.ds = cv.take<double>(vn);
  a.rhs = cv.take<double>(vm);
  a.z = cv.take<double>(vm);
  a.dy = cv.take<double>(vm);
  a.M = cv.take<double>(moff);
  a.diag = cv.take<double>(doff);
  a.tape_cap = tape_cap;
  a.tape = tape_cap ? cv.take<double>(toff) : nullptr;
  a.active = cv.take<int>(1);
  a.go = cv.take<int>(count);
  a.fail = cv.take<int>(count);
  a.minp = cv.take<unsigned long long>(count);
  a.psi = cv.take<double>(count);
  a.arg = cv.take<long long>(count);
  {
    int max_n = 0;
    for (int i = 0; i < count; ++i) max_n = std::max(max_n, (int)n[i]);
    a.nslice = (max_n + 255) / 256;
  }
  a.dpv = cv.take<double>((long)count * a.nslice);
  a.dpi = cv.take<long long>((long)count * a.nslice);
  a.dpf = cv.take<int>((long)count * a.nslice);
  h->bufptrs = cv.take<double>(6);  // x[2], y[2], s[2] pointers for get_iterate
  a.mixed = h->opt.precision == LP_PREC_MIXED;
  if (a.mixed) {
    a.refine_tol = h->opt.refine_tol;
    a.refine_max = h->opt.refine_max;
    a.switch_gap = h->opt.mixed_switch_gap;
    a.A32 = cv.take<float>(a32);
    a.M32 = cv.take<float>(m32);
    a.diag32 = cv.take<float>(doff);
    a.sd32 = cv.take<float>(vn4);
    a.r = cv.take<double>(vm);
    a.delta = cv.take<double>(vm);
    a.v = cv.take<double>(vn);
    a.fp32_mode = cv.take<int>(count);
    a.m32 = cv.take<int>(count);
    a.go64 = cv.take<int>(count);
    a.refm = cv.take<int>(count);
    a.ref_status = cv.take<int>(count);
    a.ref_steps = cv.take<int>(count);
    a.ref_prev = cv.take<double>(count);
  }
  if (tape_cap) {
    BatchAdj& g = h->adj;
    g.xb = cv.take<double>(vn);
    g.yb = cv.take<double>(vm);
    g.sb = cv.take<double>(vn);
    g.dsb = cv.take<double>(vn);
    g.db = cv.take<double>(vn);
    g.dyb = cv.take<double>(vm);
    g.lam = cv.take<double>(vm);
    g.h = cv.take<double>(vn);
    g.rdb = cv.take<double>(vn);
    g.bbar = cv.take<double>(vm);
    g.cbar = cv.take<double>(vn);
    g.err = cv.take<int>(1);
    g.Abar = nullptr;
    g.sm = vm;
    g.sn = vn;
    g.max_n = 0;
    for (int i = 0; i < count; ++i) g.max_n = std::max(g.max_n, (int)n[i]);
    g.ufac = cv.take<double>((long)tape_cap * 3 * vm);
    g.vfac = cv.take<double>((long)tape_cap * 3 * vn);
  }
}

}  // namespace

extern "C" {

lp_status lp_batch_workspace_size(int32_t count, const int64_t* m, const int64_t* n,
                                  const lp_options* opt, size_t* bytes) {
  if (!bytes) return LP_ERR_INVALID_ARG;
  if (!batch_shapes_ok(count, m, n)) return LP_ERR_SHAPE;
  lp_options o;
  lp_options_default(&o);
  if (opt) o = *opt;
  if (!(o.alpha > 0.0 && o.alpha < 1.0) || o.tape_capacity < 0) return LP_ERR_INVALID_ARG;
  if (o.precision != LP_PREC_FP64 && o.precision != LP_PREC_MIXED) return LP_ERR_INVALID_ARG;
  if (o.method != LP_METHOD_AFFINE) return LP_ERR_INVALID_ARG;
  // mixed precision: the single-LP rules, no tape (the reverse sweep
  // recomputes FP64 steps), at most kMaxBatchRefine corrections (each is
  // three launches of every captured iteration)
  if (o.precision == LP_PREC_MIXED &&
      (!(o.refine_tol >= 0) || o.refine_max < 0 || o.refine_max > kMaxBatchRefine ||
       !(o.mixed_switch_gap >= 0) || o.tape_capacity != 0))
    return LP_ERR_INVALID_ARG;
  if (o.solver != LP_SOLVER_CHOLESKY || o.reserved != 0 || o.reserved2 != 0) return LP_ERR_INVALID_ARG;
  if (o.batch_tile != 0 && o.batch_tile != 32 && o.batch_tile != 64 && o.batch_tile != 128)
    return LP_ERR_INVALID_ARG;
  if (o.batch_graph_iters < 0 || o.batch_graph_iters > 16) return LP_ERR_INVALID_ARG;
  lp_batch h;
  h.count = count;
  h.opt = o;
  Carver cv(nullptr);
  carve_batch(&h, m, n, cv);
  *bytes = (cv.off + kAlign - 1) / kAlign * kAlign;
  return LP_OK;
}

lp_status lp_batch_setup(lp_batch** out, int32_t count, const int64_t* m, const int64_t* n,
                         const double* A_packed, const int64_t* a_off, const double* b,
                         const double* c, const double* x0, const double* y0,
                         const double* s0, const int64_t* v_off_m, const int64_t* v_off_n,
                         const lp_options* opt, void* workspace, size_t ws_bytes,
                         lp_stream_t stream) {
  if (!out) return LP_ERR_INVALID_ARG;
  *out = nullptr;
  size_t need = 0;
  lp_status st = lp_batch_workspace_size(count, m, n, opt, &need);
  if (st != LP_OK) return st;
  if (!A_packed || !a_off || !b || !c || !x0 || !y0 || !s0 || !v_off_m || !v_off_n)
    return LP_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < need || ((uintptr_t)workspace % kAlign) != 0)
    return LP_ERR_WORKSPACE;
  lp_batch* h = new (std::nothrow) lp_batch();
  if (!h) return LP_ERR_INVALID_ARG;
  h->count = count;
  lp_options_default(&h->opt);
  if (opt) h->opt = *opt;
  h->st = reinterpret_cast<hipStream_t>(stream);
  Carver cv(workspace);
  carve_batch(h, m, n, cv);
  for (int i = 0; i < count; ++i) h->lps_h[i].a_off = a_off[i];
  // Descriptors (and every per-LP device array indexed like them) in
  // decreasing order of normal-matrix work m^2 n: the per-LP kernels hand
  // out their workgroups in descriptor order, so the longest start first
  // instead of forming a tail.  Pool offsets stay in the caller's order;
  // statuses go back through `order`.
  h->order.resize(count);
  for (int i = 0; i < count; ++i) h->order[i] = i;
  auto work = [&](int i) { return (double)m[i] * (double)m[i] * (double)n[i]; };
  std::stable_sort(h->order.begin(), h->order.end(),
                   [&](int x, int y) { return work(x) > work(y); });
  {
    std::vector<BatchLP> by_slot(count);
    for (int k = 0; k < count; ++k) by_slot[k] = h->lps_h[h->order[k]];
    h->lps_h.swap(by_slot);
  }
  BatchArgs& a = h->args;
  a.A = A_packed;
  a.lps = h->lps;
  a.state = h->state;
  a.tile = h->opt.batch_tile;  // 0: per-LP tile edges (the launchers' choice)
  h->graph_iters = h->opt.batch_graph_iters ? h->opt.batch_graph_iters : kItersPerGraph;
  a.alpha = h->opt.alpha;
  for (int i = 0; i < count; ++i) {
    h->max_m = std::max(h->max_m, (int)m[i]);
    h->max_tiles = std::max(h->max_tiles, (int)(((m[i] + 63) / 64) * ((n[i] + 63) / 64)));
  }
  hipStream_t s = h->st;
  std::vector<long long> uvm(count), uvn(count);
  for (int k = 0; k < count; ++k) {
    uvm[k] = v_off_m[h->order[k]];
    uvn[k] = v_off_n[h->order[k]];
  }
  long long* d_uvm = h->uvm;
  long long* d_uvn = h->uvn;
  hipError_t e =
      hipMemcpyAsync(h->lps, h->lps_h.data(), sizeof(BatchLP) * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_uvm, uvm.data(), sizeof(long long) * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_uvn, uvn.data(), sizeof(long long) * count, hipMemcpyHostToDevice, s);
  double* ptrs[6] = {a.x[0], a.x[1], a.y[0], a.y[1], a.s[0], a.s[1]};
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->bufptrs, ptrs, sizeof(ptrs), hipMemcpyHostToDevice, s);
  std::vector<int> flags(count, 0);
  if (e == hipSuccess) {
    launch_fill_i32(s, h->flags, 0, count);
    hipLaunchKernelGGL(k_batch_gather, dim3(count), dim3(256), 0, s, count, h->lps, d_uvm, d_uvn,
                       b, c, x0, y0, s0, A_packed, const_cast<double*>(a.b),
                       const_cast<double*>(a.c), a.x[0], a.y[0], a.s[0], h->flags);
    e = hipMemcpyAsync(flags.data(), h->flags, sizeof(int) * count, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    delete h;
    return LP_ERR_DEVICE;
  }
  for (int i = 0; i < count; ++i) {
    if (flags[i] & 1) st = LP_ERR_INVALID_ARG;
    else if ((flags[i] & 2) && st == LP_OK) st = LP_ERR_NOT_INTERIOR;
  }
  if (st != LP_OK) {
    delete h;
    return st;
  }
  hipLaunchKernelGGL(k_batch_init_state, dim3((count + 255) / 256), dim3(256), 0, s, count,
                     h->state);
  launch_batch_setup(s, count, h->lps, h->state, A_packed, a.c, a.x[0], a.y[0], a.s[0],
                     a.rd[0]);
  if (a.mixed) {
    launch_bmix_setup(s, count, h->max_m, h->lps, A_packed, a.A32);
    launch_fill_i32(s, a.fp32_mode, 1, count);
  }
  e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    delete h;
    return LP_ERR_DEVICE;
  }
  *out = h;
  return LP_OK;
}

// Move the still-active LPs to the first descriptor slots (relative order
// kept, so the largest still start first) and return their number and
// largest m.  Descriptors, states, the slot -> caller map and (mixed
// precision) the FP32-factor flags move together; every other per-LP array
// is either addressed through the descriptor or rebuilt at the start of
// each iteration.
static hipError_t compact_active(lp_batch* h, int cur_count, int* active_out, int* max_m_out) {
  hipStream_t s = h->st;
  std::vector<BatchState> st(cur_count);
  hipError_t e = hipMemcpyAsync(st.data(), h->state, sizeof(BatchState) * cur_count,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  std::vector<int> perm;
  perm.reserve(cur_count);
  for (int k = 0; k < cur_count; ++k)
    if (st[k].status == LP_OK) perm.push_back(k);
  const int active = (int)perm.size();
  for (int k = 0; k < cur_count; ++k)
    if (st[k].status != LP_OK) perm.push_back(k);
  std::vector<BatchLP> lps(cur_count);
  std::vector<BatchState> st2(cur_count);
  std::vector<int> ord(cur_count);
  int mm = 0;
  for (int k = 0; k < cur_count; ++k) {
    lps[k] = h->lps_h[perm[k]];
    st2[k] = st[perm[k]];
    ord[k] = h->order[perm[k]];
    if (k < active) mm = std::max(mm, lps[k].m);
  }
  std::copy(lps.begin(), lps.end(), h->lps_h.begin());
  std::copy(ord.begin(), ord.end(), h->order.begin());
  // the FP32-factor flag of a mixed batch is per LP and persistent: it moves too
  std::vector<int> f32(cur_count), f32p(cur_count);
  int* f32d = h->args.fp32_mode;
  if (f32d) {
    e = hipMemcpyAsync(f32.data(), f32d, sizeof(int) * cur_count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int k = 0; k < cur_count; ++k) f32p[k] = f32[perm[k]];
    e = hipMemcpyAsync(f32d, f32p.data(), sizeof(int) * cur_count, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
  }
  e = hipMemcpyAsync(h->lps, h->lps_h.data(), sizeof(BatchLP) * cur_count, hipMemcpyHostToDevice,
                     s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->state, st2.data(), sizeof(BatchState) * cur_count,
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  *active_out = active;
  *max_m_out = mm;
  return e;
}

// Capture graph_iters iterations of the first `count` descriptor slots into
// one graph (nothing on the legacy default stream, which cannot be captured:
// there the launches are issued directly).
static hipError_t capture_iterations(lp_batch* h, const BatchArgs& a, int max_m,
                                     hipGraph_t* graph, hipGraphExec_t* exec) {
  *graph = nullptr;
  *exec = nullptr;
  if (h->st == nullptr) return hipSuccess;
  hipError_t e = hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int k = 0; k < h->graph_iters; ++k) launch_batch_step(h->st, a, max_m, -1, nullptr);
    e = hipStreamEndCapture(h->st, graph);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
  return e;
}

lp_status lp_batch_solve(lp_batch* h, double gap_tol, int32_t max_iter, int32_t* status,
                         int32_t* iters, int32_t* n_converged) {
  if (!h || max_iter < 0 || !(gap_tol >= 0)) return LP_ERR_INVALID_ARG;
  hipStream_t s = h->st;
  BatchArgs a = h->args;
  a.tol = gap_tol;
  a.max_iter = max_iter;
  // graph_iters iterations per replayed graph.  When the LPs still running
  // are at most half of those launched for, they are moved to the first
  // slots and the graph is captured again for them alone: the launches then
  // cover fewer LPs, and only as many panel steps as the largest of them
  // needs, so the tail of a ragged batch stops paying for finished LPs.
  int cur_count = h->count, cur_max_m = h->max_m;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = capture_iterations(h, a, cur_max_m, &graph, &exec);
  int launches = 0;
  const int max_launches = max_iter / h->graph_iters + 2;
  while (e == hipSuccess) {
    if (exec) {
      e = hipGraphLaunch(exec, s);
    } else {
      for (int k = 0; k < h->graph_iters; ++k) launch_batch_step(s, a, cur_max_m, -1, nullptr);
      e = hipGetLastError();
    }
    int active = 0;
    if (e == hipSuccess)
      e = hipMemcpyAsync(&active, a.active, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ++launches;
    if (e != hipSuccess || active == 0 || launches > max_launches) break;
    bool recapture = false;
    if (a.mixed) {
      // once no LP may use the FP32 factor any more, the iteration drops
      // the FP32 and refinement launches
      std::vector<int> f32(cur_count);
      e = hipMemcpyAsync(f32.data(), a.fp32_mode, sizeof(int) * cur_count,
                         hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) break;
      if (std::none_of(f32.begin(), f32.end(), [](int v) { return v != 0; })) {
        a.mixed = 0;
        recapture = true;
      }
    }
    if (2 * active <= cur_count && cur_count > kCompactMin) {
      int n_act = 0, mm = 0;
      e = compact_active(h, cur_count, &n_act, &mm);
      if (e != hipSuccess) break;
      if (n_act == 0) break;
      cur_count = n_act;
      cur_max_m = mm;
      a.count = cur_count;
      recapture = true;
    }
    if (recapture) {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      e = capture_iterations(h, a, cur_max_m, &graph, &exec);
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return LP_ERR_DEVICE;
  std::vector<BatchState> states(h->count);
  e = hipMemcpyAsync(states.data(), h->state, sizeof(BatchState) * h->count,
                     hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return LP_ERR_DEVICE;
  int conv = 0;
  h->max_iters_run = 0;
  for (int k = 0; k < h->count; ++k) {
    const int i = h->order[k];  // slot k holds the caller's LP i
    h->max_iters_run = std::max(h->max_iters_run, states[k].iters);
    int stt = states[k].status;
    if (stt == LP_OK) stt = LP_MAX_ITER;  // never reached with max_launches above
    if (status) status[i] = stt;
    if (iters) iters[i] = states[k].iters;
    conv += (stt == LP_CONVERGED || stt == LP_OPTIMAL_PSI1);
  }
  if (n_converged) *n_converged = conv;
  return LP_OK;
}

lp_status lp_batch_iterate(lp_batch* h, double gap_tol, int32_t* status, lp_iter_info* info) {
  if (!h || !(gap_tol >= 0)) return LP_ERR_INVALID_ARG;
  hipStream_t s = h->st;
  BatchArgs a = h->args;
  a.tol = gap_tol;
  a.max_iter = INT_MAX;  // no iteration limit: the caller drives the loop
  const int count = h->count;
  std::vector<BatchState> before(count), after(count);
  std::vector<unsigned long long> minp(count);
  hipError_t e = hipMemcpyAsync(before.data(), h->state, sizeof(BatchState) * count,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) {
    launch_batch_step(s, a, h->max_m, -1, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(after.data(), h->state, sizeof(BatchState) * count,
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(minp.data(), a.minp, sizeof(unsigned long long) * count,
                       hipMemcpyDeviceToHost, s);
  std::vector<int> rst(count, 3), rsteps(count, 0);
  if (a.mixed && e == hipSuccess)
    e = hipMemcpyAsync(rst.data(), a.ref_status, sizeof(int) * count, hipMemcpyDeviceToHost, s);
  if (a.mixed && e == hipSuccess)
    e = hipMemcpyAsync(rsteps.data(), a.ref_steps, sizeof(int) * count, hipMemcpyDeviceToHost,
                       s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return LP_ERR_DEVICE;
  for (int k = 0; k < count; ++k) {
    const int i = h->order[k];  // slot k holds the caller's LP i
    const BatchState& B = before[k];
    const BatchState& S = after[k];
    h->max_iters_run = std::max(h->max_iters_run, S.iters);
    if (status) status[i] = S.status;
    if (!info) continue;
    lp_iter_info& o = info[i];
    // a step was taken when the iteration count moved, or when the step
    // itself ended the run (a rejected step leaves the count unchanged)
    const bool ran = B.status == LP_OK && !(S.status == LP_CONVERGED && S.iters == B.iters);
    // psi, t and argmax belong to this call's step when it was taken or
    // undone (LP_ERR_LOST_INTERIOR); an earlier stop leaves them stale
    const bool stepped = ran && (S.iters == B.iters + 1 || S.status == LP_ERR_LOST_INTERIOR);
    o.k = ran ? B.iters : -1;
    o.status = S.status;
    o.gap_before = B.gap;
    o.gap_after = S.gap;
    o.psi = ran ? S.last_psi : 0.0;
    o.t = stepped ? S.last_t : 0.0;
    o.argmax = stepped ? S.last_argmax : -1;
    double mp;
    std::memcpy(&mp, &minp[k], sizeof(double));
    o.min_pivot = ran ? mp : 0.0;
    // FP32 factor when its refinement converged (status 1), else FP64
    const bool used32 = ran && rst[k] == 1;
    o.precision_used = used32 ? LP_PREC_MIXED : LP_PREC_FP64;
    o.refine_steps = ran && rst[k] != 3 ? rsteps[k] : 0;
    o.refine_resid = 0.0;
  }
  return LP_OK;
}

lp_status lp_batch_get_iterate(const lp_batch* h, double* x, double* y, double* s) {
  if (!h) return LP_ERR_INVALID_ARG;
  double* const* p = reinterpret_cast<double* const*>(h->bufptrs);
  hipLaunchKernelGGL(k_batch_copy_cur, dim3(h->count), dim3(256), 0, h->st, h->count, h->lps,
                     h->state, p, p + 2, p + 4, x, y, s);
  return hipGetLastError() == hipSuccess ? LP_OK : LP_ERR_DEVICE;
}

lp_status lp_batch_backward(lp_batch* h, const double* xbar_K, const double* ybar_K,
                            const double* sbar_K, double* Abar, double* bbar, double* cbar,
                            double* x0bar, double* y0bar, double* s0bar) {
  if (!h || !xbar_K) return LP_ERR_INVALID_ARG;
  BatchArgs a = h->args;
  if (!a.tape || h->max_iters_run > a.tape_cap) return LP_ERR_NO_TAPE;
  hipStream_t s = h->st;
  BatchAdj g = h->adj;
  g.Abar = Abar;
  launch_copy(s, g.xb, xbar_K, h->sum_n);
  if (ybar_K) launch_copy(s, g.yb, ybar_K, h->sum_m);
  else launch_zero(s, g.yb, h->sum_m);
  if (sbar_K) launch_copy(s, g.sb, sbar_K, h->sum_n);
  else launch_zero(s, g.sb, h->sum_n);
  launch_zero(s, g.bbar, h->sum_m);
  launch_zero(s, g.cbar, h->sum_n);
  launch_fill_i32(s, g.err, 0, 1);
  for (int k = h->max_iters_run - 1; k >= 0; --k) launch_batch_step(s, a, h->max_m, k, &g);
  if (Abar) launch_babar(s, h->count, h->max_tiles, h->lps, h->state, g, a.tape_cap, Abar);
  if (x0bar) launch_copy(s, x0bar, g.xb, h->sum_n);
  if (y0bar) launch_copy(s, y0bar, g.yb, h->sum_m);
  if (s0bar) launch_copy(s, s0bar, g.sb, h->sum_n);
  if (bbar) launch_copy(s, bbar, g.bbar, h->sum_m);
  if (cbar) launch_copy(s, cbar, g.cbar, h->sum_n);
  int err = 0;
  hipError_t e = hipMemcpyAsync(&err, g.err, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return LP_ERR_DEVICE;
  return err ? LP_ERR_BREAKDOWN : LP_OK;
}

lp_status lp_batch_tape_row(const lp_batch* h, int32_t k, double* x, double* y, double* s) {
  if (!h) return LP_ERR_INVALID_ARG;
  if (!h->args.tape || k < 0 || k >= h->args.tape_cap) return LP_ERR_NO_TAPE;
  hipLaunchKernelGGL(k_batch_tape_row, dim3(h->count), dim3(256), 0, h->st, h->count, h->lps,
                     h->state, h->args.tape, (int)k, x, y, s);
  return hipGetLastError() == hipSuccess ? LP_OK : LP_ERR_DEVICE;
}

lp_status lp_batch_destroy(lp_batch* h) {
  delete h;
  return LP_OK;
}

}  // extern "C"
