// C ABI of libpdas: handle, workspace carving and the Section 3 loop for one
// LP.  The library never allocates device memory; every device buffer is a
// slice of the caller's workspace.  All kernels run on the handle's stream.
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "pdas_internal.h"

using namespace pdas;

namespace {

constexpr size_t kAlign = 256;

// Carves aligned slices out of a base pointer; with base == nullptr it only
// measures the total size.
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

}  // namespace

struct lp_handle {
  long m = 0, n = 0;
  lp_options opt{};
  hipStream_t st = nullptr;
  const double* A = nullptr;
  // problem copies and the double-buffered iterate
  double *b = nullptr, *c = nullptr;
  double *x[2] = {}, *y[2] = {}, *s[2] = {}, *rd[2] = {};
  int cur = 0;
  // per-iteration vectors
  double *d = nullptr, *w = nullptr, *rhs = nullptr, *z = nullptr, *dy = nullptr;
  double *dx = nullptr, *ds = nullptr, *g = nullptr, *gy = nullptr;
  // normal matrix / factor (row-major lower, ld ldm)
  double* M = nullptr;
  double* diag = nullptr;  // diagonal blocks of the factor (scratch of the Cholesky)
  long ldm = 0;
  int syrk_tile = 128, syrk_splits = 1;
  double* syrk_part = nullptr;
  size_t syrk_part_n = 0;
  // reduction scratch
  double *P1 = nullptr, *P2 = nullptr;
  int nchunks = 0;
  double* rpart = nullptr;
  long long* ipart = nullptr;
  int *zpart = nullptr, *npart = nullptr;
  int ndir = 0;
  double* gap_part = nullptr;
  int* lost_part = nullptr;
  int nstep = 0;
  int* trsv_sync = nullptr;
  int nblk = 0;
  DevInfo* info = nullptr;
  DevCheck* chk = nullptr;
  double* gap_dev = nullptr;
  // tape of start iterates [x | y | s | r_d] for the reverse sweep
  double* tape = nullptr;
  int tape_cap = 0;
  int tape_len = 0;
  // reverse-sweep buffers (carved when a tape is requested)
  double *bx = nullptr, *by = nullptr, *bs = nullptr, *brd = nullptr;
  double *xb = nullptr, *yb = nullptr, *sb = nullptr, *dsb = nullptr, *db = nullptr;
  double *dyb = nullptr, *lam = nullptr, *rdb = nullptr, *v1 = nullptr, *v2 = nullptr;
  double *v3 = nullptr, *bbar = nullptr, *cbar = nullptr, *tbar = nullptr, *tpart = nullptr;
  // host state
  int k = 0;          // directions taken since setup
  double gap = 0.0;   // x^T s of the current iterate
  // mixed precision (lp_options.precision == LP_PREC_MIXED)
  bool mixed = false;       // FP32 factor allowed at all
  bool fp32_mode = false;   // FP32 factor still in use (switches off for good)
  float* A32 = nullptr;     // FP32 copy of A
  float* M32 = nullptr;     // FP32 normal matrix / factor, row-major lower
  long ld32 = 0;
  float* sd32 = nullptr;    // sqrt(d) in FP32
  float* part32 = nullptr;
  int splits32 = 1;
  double* colsq = nullptr;  // squared column norms of A (trace of M = sum d_j c_j)
  double* rvec = nullptr;   // refinement residual
  double* delta = nullptr;  // refinement correction
  double* vtmp = nullptr;   // d o A^T dy
  double* rnorms = nullptr; // ||r||_inf, ||dy||_inf, trace(M)
  int last_prec = LP_PREC_FP64;
  int last_refine = 0;
  double last_resid = 0.0;
  // predictor-corrector (lp_options.method == LP_METHOD_PC)
  bool pc = false;
  double *dxa = nullptr, *dsa = nullptr;  // predictor direction
  double* pcq = nullptr;                  // (dx_aff o ds_aff - sigma mu) / s
  double* amin = nullptr;                 // per-block steps to the boundary
  double* mupart = nullptr;               // per-block partials of mu_aff
  // the paper's Woodbury / Egidi-Maponi solver (lp_options.solver)
  bool woodbury = false;
  double* wb_y0 = nullptr;  // (A A^T)^-1 A, columns contiguous
  double* wb_x0 = nullptr;  // (A A^T)^-1 rhs of the current iteration
  double* wb_one = nullptr; // n ones (A A^T as the normal matrix with D = I)
  // sparse A (lp_setup_csr): the caller's CSR and the CSC built from it
  bool sp = false;
  long nnz = 0;
  const int64_t* rp = nullptr;
  const int* ci = nullptr;
  const double* av = nullptr;
  int64_t* cp = nullptr;
  int *ri = nullptr, *smap = nullptr, *ssrc = nullptr, *scnt = nullptr, *scur = nullptr;
  double* cv = nullptr;
  int* sflags = nullptr;
  // phase timing (lp_options.profile)
  enum { EV_ITER0, EV_SYRK0, EV_SYRKK0, EV_SYRKK1, EV_SYRK1, EV_CHOL1, EV_TRSV1, EV_ITER1, EV_N };
  hipEvent_t ev[EV_N] = {};
  int profiling = 0;  // 0 off, 1 every phase, 2 the normal-matrix kernel alone
  // second stream and events of the grouped FP64 Cholesky (large m)
  CholAux aux;
  lp_timings tim{};
};

namespace {

struct Csc {
  int64_t* cp;
  int *ri, *map, *src, *cnt, *cur, *flags;
  double* cv;
};

void carve_csc(long n, long nnz, Carver& cv, Csc& c) {
  c.cp = cv.take<int64_t>(n + 1);
  c.ri = cv.take<int>(nnz > 0 ? nnz : 1);
  c.cv = cv.take<double>(nnz > 0 ? nnz : 1);
  c.map = cv.take<int>(nnz > 0 ? nnz : 1);
  c.src = cv.take<int>(nnz > 0 ? nnz : 1);
  c.cnt = cv.take<int>(n);
  c.cur = cv.take<int>(n);
  c.flags = cv.take<int>(4);
}

void carve_csc(lp_handle* h, Carver& cv) {
  Csc c;
  carve_csc(h->n, h->nnz, cv, c);
  h->cp = c.cp;
  h->ri = c.ri;
  h->cv = c.cv;
  h->smap = c.map;
  h->ssrc = c.src;
  h->scnt = c.cnt;
  h->scur = c.cur;
  h->sflags = c.flags;
}

void carve(lp_handle* h, Carver& cv) {
  const long m = h->m, n = h->n;
  h->b = cv.take<double>(m);
  h->c = cv.take<double>(n);
  for (int i = 0; i < 2; ++i) {
    h->x[i] = cv.take<double>(n);
    h->y[i] = cv.take<double>(m);
    h->s[i] = cv.take<double>(n);
    h->rd[i] = cv.take<double>(n);
  }
  h->d = cv.take<double>(n);
  h->w = cv.take<double>(n);
  h->rhs = cv.take<double>(m);
  h->z = cv.take<double>(m);
  h->dy = cv.take<double>(m);
  h->dx = cv.take<double>(n);
  h->ds = cv.take<double>(n);
  h->g = cv.take<double>(n);
  h->gy = cv.take<double>(n);
  h->ldm = (m + 1 + 7) / 8 * 8;  // a column beyond m: the right-hand-side row reaches (m, m)
  h->M = cv.take<double>((size_t)h->ldm * (m + 1));  // row m: the right-hand side
  h->diag = cv.take<double>(potrf_diag_elems(m));
  syrk_choose((int)m, (int)n, &h->syrk_tile, &h->syrk_splits);
  if (h->opt.syrk_tile) h->syrk_tile = h->opt.syrk_tile;
  if (h->opt.syrk_splits) {
    // a split count selects the split-K kernels
    if (h->syrk_tile == 0) h->syrk_tile = 128;
    h->syrk_splits = h->opt.syrk_splits;
  }
  h->syrk_part_n = h->sp ? 0 : syrk_part_elems((int)m, h->syrk_tile, h->syrk_splits);
  h->syrk_part = h->syrk_part_n ? cv.take<double>(h->syrk_part_n) : nullptr;
  h->nchunks = h->sp ? 1 : gemv_t_chunks(m);  // the sparse A^T product sums in full
  h->P1 = cv.take<double>((size_t)h->nchunks * n);
  h->P2 = cv.take<double>((size_t)h->nchunks * n);
  h->ndir = dir_blocks(n);
  h->rpart = cv.take<double>(h->ndir);
  h->ipart = cv.take<long long>(h->ndir);
  h->zpart = cv.take<int>(h->ndir);
  h->npart = cv.take<int>(h->ndir);
  h->nstep = step_blocks(m, n);
  h->gap_part = cv.take<double>(h->nstep > h->ndir ? h->nstep : h->ndir);
  h->lost_part = cv.take<int>(h->nstep);
  h->nblk = cdiv(m, kTB);
  h->trsv_sync = cv.take<int>(4 + 2 * h->nblk);
  h->info = cv.take<DevInfo>(1);
  h->chk = cv.take<DevCheck>(1);
  h->gap_dev = cv.take<double>(1);
  if (h->opt.precision == LP_PREC_MIXED) {
    h->ld32 = (m + 7) / 8 * 8;
    h->A32 = cv.take<float>((size_t)m * n);
    h->M32 = cv.take<float>((size_t)h->ld32 * m);
    h->sd32 = cv.take<float>(n);
    syrk_choose_f32((int)m, (int)n, &h->splits32);
    if (h->opt.syrk32_splits) h->splits32 = h->opt.syrk32_splits;
    const size_t p32 = syrk_part_elems_f32((int)m, h->splits32);
    h->part32 = p32 ? cv.take<float>(p32) : nullptr;
    h->colsq = cv.take<double>(n);
    h->rvec = cv.take<double>(m);
    h->delta = cv.take<double>(m);
    h->vtmp = cv.take<double>(n);
    h->rnorms = cv.take<double>(4);
  }
  if (h->sp) carve_csc(h, cv);
  if (h->opt.solver == LP_SOLVER_WOODBURY) {
    h->wb_y0 = cv.take<double>((size_t)m * n);
    h->wb_x0 = cv.take<double>(m);
    h->wb_one = cv.take<double>(n);
  }
  if (h->opt.method == LP_METHOD_PC) {
    h->dxa = cv.take<double>(n);
    h->dsa = cv.take<double>(n);
    h->pcq = cv.take<double>(n);
    h->amin = cv.take<double>(2 * (size_t)h->ndir);
    h->mupart = cv.take<double>(h->ndir);
  }
  h->tape_cap = h->opt.tape_capacity > 0 ? h->opt.tape_capacity : 0;
  h->tape = h->tape_cap ? cv.take<double>((size_t)(h->tape_cap + 1) * (3 * n + m)) : nullptr;
  if (h->tape_cap) {
    h->bx = cv.take<double>(n);
    h->by = cv.take<double>(m);
    h->bs = cv.take<double>(n);
    h->brd = cv.take<double>(n);
    h->xb = cv.take<double>(n);
    h->yb = cv.take<double>(m);
    h->sb = cv.take<double>(n);
    h->dsb = cv.take<double>(n);
    h->db = cv.take<double>(n);
    h->dyb = cv.take<double>(m);
    h->lam = cv.take<double>(m);
    h->rdb = cv.take<double>(n);
    h->v1 = cv.take<double>(n);
    h->v2 = cv.take<double>(n);
    h->v3 = cv.take<double>(n);
    h->bbar = cv.take<double>(m);
    h->cbar = cv.take<double>(n);
    h->tbar = cv.take<double>(1);
    h->tpart = cv.take<double>(cdiv(m > n ? m : n, 256));
  }
}

bool valid_opts(const lp_options* o) {
  if (!(o->alpha > 0.0 && o->alpha < 1.0)) return false;
  if (o->precision != LP_PREC_FP64 && o->precision != LP_PREC_MIXED) return false;
  if (o->precision == LP_PREC_MIXED &&
      (!(o->refine_tol >= 0) || o->refine_max < 0 || !(o->mixed_switch_gap >= 0)))
    return false;
  if (o->tape_capacity < 0) return false;
  if (o->syrk_tile != 0 && o->syrk_tile != 64 && o->syrk_tile != 128) return false;
  if (o->syrk_splits < 0 || o->syrk_splits > 64 || o->syrk32_splits < 0 ||
      o->syrk32_splits > 64)
    return false;
  if (o->method != LP_METHOD_AFFINE && o->method != LP_METHOD_PC) return false;
  if (o->solver != LP_SOLVER_CHOLESKY && o->solver != LP_SOLVER_WOODBURY) return false;
  if (o->reserved != 0 || o->reserved2 != 0) return false;
  if (o->batch_tile != 0 && o->batch_tile != 32 && o->batch_tile != 64 && o->batch_tile != 128)
    return false;
  if (o->batch_graph_iters < 0 || o->batch_graph_iters > 16) return false;
  if (o->solver == LP_SOLVER_WOODBURY &&
      (o->precision != LP_PREC_FP64 || o->method != LP_METHOD_AFFINE || o->tape_capacity != 0))
    return false;
  // the predictor-corrector runs in FP64 and has no reverse mode
  if (o->method == LP_METHOD_PC && (o->precision != LP_PREC_FP64 || o->tape_capacity != 0))
    return false;
  return true;
}

lp_status hip_ok(hipError_t e) { return e == hipSuccess ? LP_OK : LP_ERR_DEVICE; }

}  // namespace

extern "C" {

void lp_options_default(lp_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->alpha = 0.95;
  o->precision = LP_PREC_FP64;
  o->tape_capacity = 0;
  o->mixed_switch_gap = 1e-6;
  o->refine_tol = 0x1p-46;
  o->refine_max = 5;
}

const char* lp_status_string(int32_t s) {
  switch (s) {
    case LP_OK: return "LP_OK";
    case LP_CONVERGED: return "LP_CONVERGED";
    case LP_OPTIMAL_PSI1: return "LP_OPTIMAL_PSI1";
    case LP_OPTIMAL_ZERO_DIR: return "LP_OPTIMAL_ZERO_DIR";
    case LP_MAX_ITER: return "LP_MAX_ITER";
    case LP_ERR_INVALID_ARG: return "LP_ERR_INVALID_ARG";
    case LP_ERR_SHAPE: return "LP_ERR_SHAPE";
    case LP_ERR_NOT_INTERIOR: return "LP_ERR_NOT_INTERIOR";
    case LP_ERR_BREAKDOWN: return "LP_ERR_BREAKDOWN";
    case LP_ERR_NONPOS_PSI: return "LP_ERR_NONPOS_PSI";
    case LP_ERR_LOST_INTERIOR: return "LP_ERR_LOST_INTERIOR";
    case LP_ERR_WORKSPACE: return "LP_ERR_WORKSPACE";
    case LP_ERR_NO_TAPE: return "LP_ERR_NO_TAPE";
    case LP_ERR_DEVICE: return "LP_ERR_DEVICE";
    default: return "LP_UNKNOWN_STATUS";
  }
}

// Shape, option and workspace rules shared by the dense and the CSR setup.
static lp_status workspace_size_impl(int64_t m, int64_t n, bool sparse, int64_t nnz,
                                     const lp_options* opt, size_t* bytes) {
  if (!bytes) return LP_ERR_INVALID_ARG;
  if (m < 1 || n <= m || m > INT_MAX / 2 || n > INT_MAX / 2) return LP_ERR_SHAPE;
  if (sparse && (m > LP_CSR_MAX_M || !sp_fits(m) || nnz < 0 || nnz > INT_MAX))
    return LP_ERR_SHAPE;
  lp_options o;
  lp_options_default(&o);
  if (opt) o = *opt;
  if (!valid_opts(&o)) return LP_ERR_INVALID_ARG;
  // the sparse path: FP64 Cholesky, no tape (affine or predictor-corrector)
  if (sparse && (o.precision != LP_PREC_FP64 || o.solver != LP_SOLVER_CHOLESKY ||
                 o.tape_capacity != 0))
    return LP_ERR_INVALID_ARG;
  if (o.solver == LP_SOLVER_WOODBURY && !woodbury_fits(m, n)) return LP_ERR_SHAPE;
  lp_handle h;
  h.m = m;
  h.n = n;
  h.opt = o;
  h.sp = sparse;
  h.nnz = sparse ? nnz : 0;
  Carver cv(nullptr);
  carve(&h, cv);
  *bytes = (cv.off + kAlign - 1) / kAlign * kAlign;
  return LP_OK;
}

// Checks A's CSR on the device (structure, finiteness) and builds the CSC;
// synchronises.  LP_ERR_INVALID_ARG for a bad CSR.
static lp_status csr_prepare(hipStream_t s, long m, long n, long nnz, const int64_t* rp,
                             const int* ci, const double* v, int* flags, int64_t* cp, int* ri,
                             double* cv, int* src, int* map, int* cnt, int* cur) {
  launch_fill_i32(s, flags, 0, 4);
  launch_sp_check(s, m, n, nnz, rp, ci, v, flags);
  int hf[4] = {};
  hipError_t e = hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return LP_ERR_DEVICE;
  if (hf[0]) return LP_ERR_INVALID_ARG;
  e = sp_prepare();
  if (e != hipSuccess) return LP_ERR_DEVICE;
  launch_sp_transpose(s, m, n, nnz, rp, ci, v, cnt, cur, cp, ri, cv, src, map);
  e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? LP_OK : LP_ERR_DEVICE;
}

// A^T v1 (and A^T v2) into the handle's partial sums P1 (P2), dense or CSC.
static void apply_At(lp_handle* h, const double* v1, const double* v2) {
  if (h->sp)
    launch_sp_gemv_t(h->st, h->n, h->nnz, h->cp, h->ri, h->cv, v1, v2, h->P1, v2 ? h->P2 : nullptr);
  else
    launch_gemv_t(h->st, h->m, h->n, h->A, v1, v2, h->P1, v2 ? h->P2 : nullptr);
}

// out = base + sign * A w, dense or CSR.
static void apply_A(lp_handle* h, const double* w, const double* base, double* out,
                    double sign = 1.0) {
  if (h->sp) launch_sp_gemv_n(h->st, h->m, h->nnz, h->rp, h->ci, h->av, w, base, out, sign);
  else launch_gemv_n(h->st, h->m, h->n, h->A, w, base, out, sign);
}

// Everything after the carve: device validation, copies, r_d, gap, the
// Woodbury preparation and the profiling events.  Deletes h on error.
static lp_status setup_finish(lp_handle* h, const double* b, const double* c, const double* x0,
                              const double* y0, const double* s0) {
  const long m = h->m, n = h->n;
  hipStream_t s = h->st;
  lp_status st = LP_OK;
  // validation on the device: finiteness and interior start
  hipError_t e = hipMemsetAsync(h->chk, 0, sizeof(DevCheck), s);
  if (e == hipSuccess) {
    launch_check_inputs(s, m, n, h->A, b, c, x0, y0, s0, h->chk);  // A null when sparse
    DevCheck chk{};
    e = hipMemcpyAsync(&chk, h->chk, sizeof(chk), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess && chk.nonfinite) st = LP_ERR_INVALID_ARG;
    else if (e == hipSuccess && chk.nonpos) st = LP_ERR_NOT_INTERIOR;
  }
  if (e != hipSuccess) st = LP_ERR_DEVICE;
  if (st == LP_OK && h->sp)
    st = csr_prepare(s, m, n, h->nnz, h->rp, h->ci, h->av, h->sflags, h->cp, h->ri, h->cv,
                     h->ssrc, h->smap, h->scnt, h->scur);
  if (st != LP_OK) {
    delete h;
    return st;
  }
  // copies of the problem and the start point
  launch_copy(s, h->b, b, m);
  launch_copy(s, h->c, c, n);
  launch_copy(s, h->x[0], x0, n);
  launch_copy(s, h->y[0], y0, m);
  launch_copy(s, h->s[0], s0, n);
  h->cur = 0;
  launch_fill_i32(s, h->trsv_sync, 0, 4 + 2 * h->nblk);
  h->pc = h->opt.method == LP_METHOD_PC;
  if (h->opt.precision == LP_PREC_MIXED) {
    h->mixed = true;
    h->fp32_mode = true;
    launch_to_f32(s, m * n, h->A, h->A32);
    launch_colsq(s, m, n, h->A, h->colsq);
  }
  // r_d = c - A^T y0 - s0
  apply_At(h, h->y[0], nullptr);
  launch_dual_resid(s, m, n, h->P1, h->nchunks, h->c, h->s[0], h->rd[0]);
  launch_gap(s, n, h->x[0], h->s[0], h->gap_part, h->gap_dev);
  double gap = 0;
  e = hipMemcpyAsync(&gap, h->gap_dev, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    delete h;
    return LP_ERR_DEVICE;
  }
  h->gap = gap;
  h->k = 0;
  h->tape_len = 0;
  if (h->opt.solver == LP_SOLVER_WOODBURY) {
    // once: the factor of A A^T (kept in M) and (A A^T)^-1 A
    h->woodbury = true;
    e = woodbury_prepare();
    if (e == hipSuccess) {
      launch_wb_fill(s, n, 1.0, h->wb_one);
      launch_iter_begin(s, h->info, h->trsv_sync, h->nblk);
      launch_syrk_f64(s, (int)m, (int)n, h->A, n, h->wb_one, h->M, h->ldm, false, h->syrk_tile,
                      h->syrk_splits, h->syrk_part);
      launch_potrf_f64(s, (int)m, (int)m, h->M, h->ldm, h->info, h->diag, &h->aux);
      launch_wb_cols(s, (int)m, (int)n, h->M, h->ldm, h->A, h->wb_y0);
      DevInfo di{};
      e = hipMemcpyAsync(&di, h->info, sizeof(di), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess && di.chol_fail != INT_MAX) {
        delete h;
        return LP_ERR_BREAKDOWN;  // A A^T not positive definite: A rank-deficient
      }
    }
    if (e != hipSuccess) {
      delete h;
      return LP_ERR_DEVICE;
    }
  }
  if (chol_grouped((int)m)) {
    if (hipStreamCreateWithFlags(&h->aux.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->aux.ev_main, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->aux.ev_aux, hipEventDisableTiming) != hipSuccess) {
      lp_destroy(h);
      return LP_ERR_DEVICE;
    }
  }
  if (h->opt.profile) {
    h->profiling = h->opt.profile == 2 ? 2 : 1;
    for (int i = 0; i < lp_handle::EV_N; ++i) {
      if (hipEventCreate(&h->ev[i]) != hipSuccess) {
        lp_destroy(h);
        return LP_ERR_DEVICE;
      }
    }
  }
  return LP_OK;
}

lp_status lp_workspace_size(int64_t m, int64_t n, const lp_options* opt, size_t* bytes) {
  return workspace_size_impl(m, n, false, 0, opt, bytes);
}

lp_status lp_workspace_size_csr(int64_t m, int64_t n, int64_t nnz, const lp_options* opt,
                                size_t* bytes) {
  return workspace_size_impl(m, n, true, nnz, opt, bytes);
}

lp_status lp_setup(lp_handle** out, int64_t m, int64_t n, const double* A, const double* b,
                   const double* c, const double* x0, const double* y0, const double* s0,
                   const lp_options* opt, void* workspace, size_t ws_bytes, lp_stream_t stream) {
  if (!out) return LP_ERR_INVALID_ARG;
  *out = nullptr;
  size_t need = 0;
  lp_status st = lp_workspace_size(m, n, opt, &need);
  if (st != LP_OK) return st;
  if (!A || !b || !c || !x0 || !y0 || !s0) return LP_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < need || ((uintptr_t)workspace % kAlign) != 0)
    return LP_ERR_WORKSPACE;
  lp_handle* h = new (std::nothrow) lp_handle();
  if (!h) return LP_ERR_INVALID_ARG;
  h->m = m;
  h->n = n;
  lp_options_default(&h->opt);
  if (opt) h->opt = *opt;
  h->st = reinterpret_cast<hipStream_t>(stream);
  h->A = A;
  Carver cv(workspace);
  carve(h, cv);
  st = setup_finish(h, b, c, x0, y0, s0);
  if (st == LP_OK) *out = h;
  return st;
}

lp_status lp_setup_csr(lp_handle** out, int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                       const int32_t* col_idx, const double* vals, const double* b,
                       const double* c, const double* x0, const double* y0, const double* s0,
                       const lp_options* opt, void* workspace, size_t ws_bytes,
                       lp_stream_t stream) {
  if (!out) return LP_ERR_INVALID_ARG;
  *out = nullptr;
  size_t need = 0;
  lp_status st = lp_workspace_size_csr(m, n, nnz, opt, &need);
  if (st != LP_OK) return st;
  if (!row_ptr || (nnz > 0 && (!col_idx || !vals)) || !b || !c || !x0 || !y0 || !s0)
    return LP_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < need || ((uintptr_t)workspace % kAlign) != 0)
    return LP_ERR_WORKSPACE;
  lp_handle* h = new (std::nothrow) lp_handle();
  if (!h) return LP_ERR_INVALID_ARG;
  h->m = m;
  h->n = n;
  lp_options_default(&h->opt);
  if (opt) h->opt = *opt;
  h->st = reinterpret_cast<hipStream_t>(stream);
  h->sp = true;
  h->nnz = nnz;
  h->rp = row_ptr;
  h->ci = col_idx;
  h->av = vals;
  Carver cv(workspace);
  carve(h, cv);
  st = setup_finish(h, b, c, x0, y0, s0);
  if (st == LP_OK) *out = h;
  return st;
}

static void record_tape(lp_handle* h) {
  if (!h->tape || h->tape_len > h->tape_cap) return;
  const long m = h->m, n = h->n, row = 3 * n + m;
  double* r = h->tape + (size_t)h->tape_len * row;
  launch_copy(h->st, r, h->x[h->cur], n);
  launch_copy(h->st, r + n, h->y[h->cur], m);
  launch_copy(h->st, r + n + m, h->s[h->cur], n);
  launch_copy(h->st, r + 2 * n + m, h->rd[h->cur], n);
  h->tape_len++;
}

// Enqueue one iteration (FP64) from the current iterate into the other buffer.
static void mark(lp_handle* h, int i) {
  if (h->profiling == 1 ||
      (h->profiling == 2 && (i == lp_handle::EV_SYRKK0 || i == lp_handle::EV_SYRKK1)))
    (void)hipEventRecord(h->ev[i], h->st);
}

// FP64 direction: normal matrix, Cholesky, the two triangular solves.
static void solve_fp64(lp_handle* h) {
  const long m = h->m, n = h->n;
  hipStream_t s = h->st;
  if (h->sp) {
    mark(h, lp_handle::EV_SYRKK0);
    launch_sp_syrk(s, m, h->rp, h->ci, h->av, h->cp, h->ri, h->cv, h->smap, h->d, h->M, h->ldm);
    mark(h, lp_handle::EV_SYRKK1);
  } else {
    launch_syrk_f64(s, (int)m, (int)n, h->A, n, h->d, h->M, h->ldm, false, h->syrk_tile,
                    h->syrk_splits, h->syrk_part,
                    h->profiling ? h->ev[lp_handle::EV_SYRKK0] : nullptr,
                    h->profiling ? h->ev[lp_handle::EV_SYRKK1] : nullptr);
  }
  mark(h, lp_handle::EV_SYRK1);
  // rhs rides along as row m of the factorization: it leaves as z = L^-1 rhs
  double* zrow = h->M + (size_t)m * h->ldm;
  launch_copy(s, zrow, h->rhs, m);
  launch_potrf_f64(s, (int)m + 1, (int)m, h->M, h->ldm, h->info, h->diag, &h->aux);
  mark(h, lp_handle::EV_CHOL1);
  launch_trsv_bwd(s, (int)m, h->M, h->ldm, zrow, h->dy, h->trsv_sync, h->info);
  h->last_prec = LP_PREC_FP64;
}

// The paper's Section 5 direction: x0 = (A A^T)^-1 rhs with the factor of
// A A^T kept in M since setup, then the Egidi-Maponi recurrence over the n
// rank-one terms (d_l - 1) a_l a_l^T.
static void solve_woodbury(lp_handle* h) {
  const long m = h->m, n = h->n;
  hipStream_t s = h->st;
  // no normal matrix in this solver: its phase events are recorded empty,
  // so that every event of the iteration's timing has been recorded
  mark(h, lp_handle::EV_SYRKK0);
  mark(h, lp_handle::EV_SYRKK1);
  mark(h, lp_handle::EV_SYRK1);
  launch_trsv_fwd(s, (int)m, h->M, h->ldm, h->rhs, h->z, h->trsv_sync, h->info);
  launch_trsv_bwd(s, (int)m, h->M, h->ldm, h->z, h->wb_x0, h->trsv_sync, h->info);
  launch_woodbury(s, (int)m, (int)n, h->A, h->d, h->wb_y0, h->wb_x0, h->dy, h->info);
  mark(h, lp_handle::EV_CHOL1);
  h->last_prec = LP_PREC_FP64;
}

// Read the device info record (synchronises the stream).
static bool read_info(lp_handle* h, DevInfo* di) {
  hipError_t e = hipMemcpyAsync(di, h->info, sizeof(*di), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  return e == hipSuccess;
}

// Mixed precision direction: FP32 normal matrix (sqrt(D) column scaling) and
// FP32 Cholesky on the matrix cores, the factor widened to FP64 for the
// triangular solves, then FP64 iterative refinement on the matrix-free
// residual r = rhs - A (d o (A^T dy)):  delta = L^-T L^-1 r,  dy += delta.
// Stopping rule on the corrections: with q_i = ||delta_i|| / ||delta_{i-1}||
// (the observed contraction), refinement has converged when
//   ||delta_i|| / ||dy|| <= refine_tol   or   (q_i < 1/2 and
//   ||delta_i|| q_i / (1 - q_i) / ||dy|| <= refine_tol)
// (the second term bounds the error that remains after a geometric series
// of further corrections).  An FP32 pivot failure, q_i >= 1/2 (stagnation),
// or refine_max corrections without convergence fall back to the FP64 solve
// and stay in FP64.  Returns false when a HIP call failed.
static bool solve_mixed(lp_handle* h, bool* ok) {
  const long m = h->m, n = h->n;
  hipStream_t s = h->st;
  *ok = false;
  h->last_refine = 0;
  h->last_resid = 0.0;
  if (!launch_syrk_f32(s, (int)m, (int)n, h->A32, n, h->sd32, h->M32, h->ld32, false,
                       h->splits32, h->part32,
                       h->profiling ? h->ev[lp_handle::EV_SYRKK0] : nullptr,
                       h->profiling ? h->ev[lp_handle::EV_SYRKK1] : nullptr))
    return true;  // shapes the FP32 kernel does not take: FP64
  mark(h, lp_handle::EV_SYRK1);
  launch_potrf_f32(s, (int)m, h->M32, h->ld32, h->info, reinterpret_cast<float*>(h->diag));
  mark(h, lp_handle::EV_CHOL1);
  DevInfo di;
  if (!read_info(h, &di)) return false;
  if (di.chol_fail != INT_MAX) return true;
  launch_lower_f32_to_f64(s, m, h->M32, h->ld32, h->M, h->ldm);
  launch_trsv_fwd(s, (int)m, h->M, h->ldm, h->rhs, h->z, h->trsv_sync, h->info);
  launch_trsv_bwd(s, (int)m, h->M, h->ldm, h->z, h->dy, h->trsv_sync, h->info);
  double prev = INFINITY;
  for (int step = 0; step < h->opt.refine_max; ++step) {
    launch_gemv_t(s, m, n, h->A, h->dy, nullptr, h->P1, nullptr);
    launch_scale_partials(s, n, h->P1, h->nchunks, h->d, h->vtmp);
    launch_gemv_n(s, m, n, h->A, h->vtmp, h->rhs, h->rvec, -1.0);
    launch_fill_i32(s, h->trsv_sync, 0, 4 + 2 * h->nblk);
    launch_trsv_fwd(s, (int)m, h->M, h->ldm, h->rvec, h->z, h->trsv_sync, h->info);
    launch_trsv_bwd(s, (int)m, h->M, h->ldm, h->z, h->delta, h->trsv_sync, h->info);
    launch_axpy(s, m, h->delta, h->dy);
    // ||delta||_inf, ||dy||_inf (after the update)
    launch_refine_norms(s, m, n, h->delta, h->dy, h->d, h->colsq, h->rnorms);
    double nr[4];
    hipError_t e = hipMemcpyAsync(nr, h->rnorms, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return false;
    if (!read_info(h, &di)) return false;
    if (di.trsv_err) return true;
    h->last_refine = step + 1;
    const double dn = nr[0], yn = nr[1];
    if (!std::isfinite(dn) || !std::isfinite(yn) || !(yn > 0)) break;
    const double rel = dn / yn;
    h->last_resid = rel;
    if (rel <= h->opt.refine_tol) {
      *ok = true;
      break;
    }
    if (step > 0) {
      const double q = dn / prev;
      if (!(q < 0.5)) break;  // stagnation
      const double rest = rel * q / (1.0 - q);
      if (rest <= h->opt.refine_tol) {
        h->last_resid = rest;
        *ok = true;
        break;
      }
    }
    prev = dn;
  }
  if (*ok) h->last_prec = LP_PREC_MIXED;
  return true;
}

// One predictor-corrector iteration (LP_METHOD_PC): the Section 3 direction
// as predictor (normal matrix, factor, the right-hand side carried through
// the factorization), its steps to the boundary and the centring parameter,
// then the corrector solve with the same factor, the corrector direction and
// the step, from the current iterate into the other buffer.
static void enqueue_pc_iteration(lp_handle* h) {
  const long m = h->m, n = h->n;
  hipStream_t s = h->st;
  const int cur = h->cur, nxt = cur ^ 1;
  mark(h, lp_handle::EV_ITER0);
  launch_iter_begin(s, h->info, h->trsv_sync, h->nblk);
  launch_prep(s, n, h->x[cur], h->s[cur], h->rd[cur], h->d, h->w);
  apply_A(h, h->w, h->b, h->rhs);
  mark(h, lp_handle::EV_SYRK0);
  solve_fp64(h);  // dy: the predictor
  apply_At(h, h->dy, h->y[cur]);
  launch_pc_aff(s, n, h->P1, h->P2, h->nchunks, h->rd[cur], h->x[cur], h->s[cur], h->d, h->dxa,
                h->dsa, h->gy, h->amin);
  launch_pc_corr(s, n, h->gap, h->amin, h->x[cur], h->s[cur], h->rd[cur], h->d, h->dxa, h->dsa,
                 h->mupart, h->pcq, h->w, h->info);
  apply_A(h, h->w, h->b, h->rhs);
  launch_fill_i32(s, h->trsv_sync, 0, 4 + 2 * h->nblk);
  launch_trsv_fwd(s, (int)m, h->M, h->ldm, h->rhs, h->z, h->trsv_sync, h->info);
  launch_trsv_bwd(s, (int)m, h->M, h->ldm, h->z, h->dy, h->trsv_sync, h->info);
  mark(h, lp_handle::EV_TRSV1);
  apply_At(h, h->dy, nullptr);
  launch_pc_dir(s, n, h->P1, h->nchunks, h->rd[cur], h->x[cur], h->s[cur], h->d, h->pcq, h->dx,
                h->ds, h->g, h->amin, h->zpart, h->npart);
  launch_pc_step(s, m, n, h->opt.alpha, h->amin, h->zpart, h->npart, h->dy, h->x[cur], h->y[cur],
                 h->s[cur], h->dx, h->ds, h->g, h->gy, h->c, h->x[nxt], h->y[nxt], h->s[nxt],
                 h->rd[nxt], h->gap_part, h->lost_part, h->info);
  launch_finish(s, h->nstep, h->gap_part, h->lost_part, h->info);
  mark(h, lp_handle::EV_ITER1);
}

// Enqueue one iteration from the current iterate into the other buffer.
static bool enqueue_iteration(lp_handle* h) {
  if (h->pc) {
    enqueue_pc_iteration(h);
    return true;
  }
  const long m = h->m, n = h->n;
  hipStream_t s = h->st;
  const int cur = h->cur, nxt = cur ^ 1;
  if (h->fp32_mode && h->gap < h->opt.mixed_switch_gap) h->fp32_mode = false;
  mark(h, lp_handle::EV_ITER0);
  launch_iter_begin(s, h->info, h->trsv_sync, h->nblk);
  launch_prep(s, n, h->x[cur], h->s[cur], h->rd[cur], h->d, h->w,
              h->fp32_mode ? h->sd32 : nullptr);
  apply_A(h, h->w, h->b, h->rhs);
  mark(h, lp_handle::EV_SYRK0);
  bool done = false;
  if (h->fp32_mode) {
    if (!solve_mixed(h, &done)) return false;
    if (!done) {
      h->fp32_mode = false;  // stay in FP64 from now on
      launch_iter_begin(s, h->info, h->trsv_sync, h->nblk);
    }
  }
  if (!done) {
    if (h->woodbury) solve_woodbury(h);
    else solve_fp64(h);
  }
  mark(h, lp_handle::EV_TRSV1);
  apply_At(h, h->dy, h->y[cur]);
  launch_dir(s, m, n, h->P1, h->P2, h->nchunks, h->rd[cur], h->x[cur], h->s[cur], h->d, h->dx,
             h->ds, h->gy, h->g, h->rpart, h->ipart, h->zpart, h->npart);
  launch_step(s, m, n, h->opt.alpha, h->ndir, h->rpart, h->ipart, h->zpart, h->npart, h->dy,
              h->x[cur], h->y[cur], h->s[cur], h->dx, h->ds, h->g, h->gy, h->c, h->x[nxt],
              h->y[nxt], h->s[nxt], h->rd[nxt], h->gap_part, h->lost_part, h->info);
  launch_finish(s, h->nstep, h->gap_part, h->lost_part, h->info);
  mark(h, lp_handle::EV_ITER1);
  return true;
}

static void accumulate_timings(lp_handle* h) {
  if (!h->profiling) return;
  float t[8] = {};
  auto el = [&](int a, int b) {
    float ms = 0;
    return hipEventElapsedTime(&ms, h->ev[a], h->ev[b]) == hipSuccess ? (double)ms : 0.0;
  };
  typedef lp_handle H;
  if (h->profiling == 2) {
    h->tim.normal_kernel_ms += el(H::EV_SYRKK0, H::EV_SYRKK1);
    h->tim.normal_launches += 1;
    h->tim.iterations += 1;
    return;
  }
  const double iter = el(H::EV_ITER0, H::EV_ITER1);
  const double syrk = el(H::EV_SYRK0, H::EV_SYRK1);
  const double syrkk = el(H::EV_SYRKK0, H::EV_SYRKK1);
  const double chol = el(H::EV_SYRK1, H::EV_CHOL1);
  const double trsv = el(H::EV_CHOL1, H::EV_TRSV1);
  (void)t;
  h->tim.iter_ms += iter;
  h->tim.normal_ms += syrk;
  h->tim.normal_kernel_ms += syrkk;
  h->tim.potrf_ms += chol;
  h->tim.trsv_ms += trsv;
  h->tim.other_ms += iter - syrk - chol - trsv;
  h->tim.iterations += 1;
  h->tim.normal_launches += 1;
}

lp_status lp_iterate(lp_handle* h, lp_iter_info* info) {
  if (!h) return LP_ERR_INVALID_ARG;
  record_tape(h);
  if (!enqueue_iteration(h)) return LP_ERR_DEVICE;
  DevInfo di;
  hipError_t e = hipMemcpyAsync(&di, h->info, sizeof(di), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return LP_ERR_DEVICE;
  accumulate_timings(h);
  const lp_status st = (lp_status)di.status;
  const bool stepped = (st == LP_OK || st == LP_OPTIMAL_PSI1);
  if (info) {
    info->k = h->k;
    info->status = st;
    info->gap_before = h->gap;
    info->gap_after = stepped ? di.gap_after : h->gap;
    info->psi = di.psi;
    info->t = di.t;
    info->argmax = di.argmax;
    info->min_pivot = di.min_pivot;
    info->precision_used = h->last_prec;
    info->refine_steps = h->last_prec == LP_PREC_MIXED ? h->last_refine : 0;
    info->refine_resid = h->last_prec == LP_PREC_MIXED ? h->last_resid : 0.0;
    info->alpha_primal = h->pc ? di.alpha_p : di.t;
    info->alpha_dual = h->pc ? di.alpha_d : di.t;
    info->sigma = h->pc ? di.sigma : 0.0;
  }
  if (stepped) {
    h->cur ^= 1;
    h->gap = di.gap_after;
    h->k++;
  } else if (h->tape_len > 0) {
    h->tape_len--;  // the recorded start of a step that did not happen
  }
  return st;
}

lp_status lp_solve(lp_handle* h, double gap_tol, int32_t max_iter, lp_result* result,
                   lp_iter_info* log) {
  if (!h || max_iter < 0 || !(gap_tol >= 0)) return LP_ERR_INVALID_ARG;
  lp_status st = LP_OK;
  int taken = 0;
  for (;;) {
    if (h->gap < gap_tol) {
      st = LP_CONVERGED;
      break;
    }
    if (taken >= max_iter) {
      st = LP_MAX_ITER;
      break;
    }
    lp_iter_info it;
    st = lp_iterate(h, &it);
    if (log && (st == LP_OK || st == LP_OPTIMAL_PSI1 || st < 0)) log[taken] = it;
    if (st == LP_OK) {
      ++taken;
      continue;
    }
    if (st == LP_OPTIMAL_PSI1) ++taken;
    break;
  }
  if (h->tape && h->tape_len <= h->tape_cap) record_tape(h);  // final iterate
  if (result) {
    result->status = st;
    result->iters = taken;
    result->gap = h->gap;
    // objectives: c^T x and b^T y (ordered block sums)
    double* tmp = h->gap_dev;
    double cx = NAN, by = NAN;
    launch_gap(h->st, h->n, h->c, h->x[h->cur], h->gap_part, tmp);
    hipError_t e = hipMemcpyAsync(&cx, tmp, sizeof(double), hipMemcpyDeviceToHost, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    launch_gap(h->st, h->m, h->b, h->y[h->cur], h->gap_part, tmp);
    if (e == hipSuccess) e = hipMemcpyAsync(&by, tmp, sizeof(double), hipMemcpyDeviceToHost, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return LP_ERR_DEVICE;
    result->primal_obj = cx;
    result->dual_obj = by;
  }
  return st;
}

lp_status lp_get_iterate(const lp_handle* h, double* x, double* y, double* s) {
  if (!h) return LP_ERR_INVALID_ARG;
  if (x) launch_copy(h->st, x, h->x[h->cur], h->n);
  if (y) launch_copy(h->st, y, h->y[h->cur], h->m);
  if (s) launch_copy(h->st, s, h->s[h->cur], h->n);
  return hip_ok(hipGetLastError());
}

lp_status lp_get_direction(const lp_handle* h, double* dx, double* dy, double* ds) {
  if (!h) return LP_ERR_INVALID_ARG;
  if (dx) launch_copy(h->st, dx, h->dx, h->n);
  if (dy) launch_copy(h->st, dy, h->dy, h->m);
  if (ds) launch_copy(h->st, ds, h->ds, h->n);
  return hip_ok(hipGetLastError());
}

lp_status lp_backward(lp_handle* h, const double* xbar_K, const double* ybar_K,
                      const double* sbar_K, double* Abar, double* bbar, double* cbar,
                      double* x0bar, double* y0bar, double* s0bar) {
  if (!h || !xbar_K) return LP_ERR_INVALID_ARG;
  if (!h->tape || h->k > h->tape_cap || h->tape_len < h->k) return LP_ERR_NO_TAPE;
  const long m = h->m, n = h->n, row = 3 * n + m;
  const int K = h->k;
  hipStream_t s = h->st;
  const int nxt = h->cur ^ 1;  // scratch outputs of the recomputed steps
  launch_copy(s, h->xb, xbar_K, n);
  if (ybar_K) launch_copy(s, h->yb, ybar_K, m);
  else launch_zero(s, h->yb, m);
  if (sbar_K) launch_copy(s, h->sb, sbar_K, n);
  else launch_zero(s, h->sb, n);
  launch_zero(s, h->bbar, m);
  launch_zero(s, h->cbar, n);
  if (Abar) launch_zero(s, Abar, m * n);
  for (int k = K - 1; k >= 0; --k) {
    const double* r = h->tape + (size_t)k * row;
    launch_copy(s, h->bx, r, n);
    launch_copy(s, h->by, r + n, m);
    launch_copy(s, h->bs, r + n + m, n);
    launch_copy(s, h->brd, r + 2 * n + m, n);
    // recompute step k exactly as the forward pass did (FP64)
    launch_iter_begin(s, h->info, h->trsv_sync, h->nblk);
    launch_prep(s, n, h->bx, h->bs, h->brd, h->d, h->w);
    launch_gemv_n(s, m, n, h->A, h->w, h->b, h->rhs);
    launch_syrk_f64(s, (int)m, (int)n, h->A, n, h->d, h->M, h->ldm, false, h->syrk_tile,
                    h->syrk_splits, h->syrk_part);
    double* zrow = h->M + (size_t)m * h->ldm;
    launch_copy(s, zrow, h->rhs, m);
    launch_potrf_f64(s, (int)m + 1, (int)m, h->M, h->ldm, h->info, h->diag, &h->aux);
    launch_trsv_bwd(s, (int)m, h->M, h->ldm, zrow, h->dy, h->trsv_sync, h->info);
    launch_gemv_t(s, m, n, h->A, h->dy, h->by, h->P1, h->P2);
    launch_dir(s, m, n, h->P1, h->P2, h->nchunks, h->brd, h->bx, h->bs, h->d, h->dx, h->ds,
               h->gy, h->g, h->rpart, h->ipart, h->zpart, h->npart);
    launch_step(s, m, n, h->opt.alpha, h->ndir, h->rpart, h->ipart, h->zpart, h->npart, h->dy,
                h->bx, h->by, h->bs, h->dx, h->ds, h->g, h->gy, h->c, h->x[nxt], h->y[nxt],
                h->s[nxt], h->rd[nxt], h->gap_part, h->lost_part, h->info);
    // reverse of step k
    launch_adj_tbar(s, m, n, h->xb, h->dx, h->sb, h->ds, h->yb, h->dy, h->tpart, h->tbar);
    launch_adj_a(s, m, n, h->opt.alpha, h->info, h->tbar, h->bx, h->bs, h->d, h->dx, h->ds,
                 h->xb, h->sb, h->yb, h->dsb, h->db, h->dyb);
    launch_gemv_n(s, m, n, h->A, h->dsb, h->dyb, h->dyb, -1.0);
    launch_fill_i32(s, h->trsv_sync, 0, 4 + 2 * h->nblk);
    launch_trsv_fwd(s, (int)m, h->M, h->ldm, h->dyb, h->z, h->trsv_sync, h->info);
    launch_trsv_bwd(s, (int)m, h->M, h->ldm, h->z, h->lam, h->trsv_sync, h->info);
    launch_gemv_t(s, m, n, h->A, h->lam, nullptr, h->P1, nullptr);
    launch_adj_b(s, m, n, h->P1, h->nchunks, h->g, h->brd, h->d, h->bx, h->bs, h->lam, h->dsb,
                 h->db, h->xb, h->sb, h->cbar, h->rdb, h->bbar, h->v1, h->v2, h->v3);
    launch_gemv_n(s, m, n, h->A, h->rdb, h->yb, h->yb, -1.0);
    if (Abar) launch_rank3(s, m, n, Abar, h->dy, h->v1, h->lam, h->v2, h->by, h->v3);
    DevInfo di;
    hipError_t e = hipMemcpyAsync(&di, h->info, sizeof(di), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return LP_ERR_DEVICE;
    if (di.chol_fail != INT_MAX) return LP_ERR_BREAKDOWN;
    if (di.trsv_err) return LP_ERR_DEVICE;
  }
  if (x0bar) launch_copy(s, x0bar, h->xb, n);
  if (y0bar) launch_copy(s, y0bar, h->yb, m);
  if (s0bar) launch_copy(s, s0bar, h->sb, n);
  if (bbar) launch_copy(s, bbar, h->bbar, m);
  if (cbar) launch_copy(s, cbar, h->cbar, n);
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? LP_OK : LP_ERR_DEVICE;
}

lp_status lp_tape_row(const lp_handle* h, int32_t k, double* x, double* y, double* s) {
  if (!h) return LP_ERR_INVALID_ARG;
  if (!h->tape || k < 0 || k >= h->tape_len) return LP_ERR_NO_TAPE;
  const long m = h->m, n = h->n;
  const double* r = h->tape + (size_t)k * (3 * n + m);
  if (x) launch_copy(h->st, x, r, n);
  if (y) launch_copy(h->st, y, r + n, m);
  if (s) launch_copy(h->st, s, r + n + m, n);
  return hip_ok(hipGetLastError());
}

lp_status lp_get_timings(const lp_handle* h, lp_timings* out) {
  if (!h || !out) return LP_ERR_INVALID_ARG;
  *out = h->tim;
  return LP_OK;
}

lp_status lp_destroy(lp_handle* h) {
  if (!h) return LP_OK;
  for (int i = 0; i < lp_handle::EV_N; ++i)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  if (h->aux.ev_main) (void)hipEventDestroy(h->aux.ev_main);
  if (h->aux.ev_aux) (void)hipEventDestroy(h->aux.ev_aux);
  if (h->aux.st) (void)hipStreamDestroy(h->aux.st);
  delete h;
  return LP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Building blocks
// ---------------------------------------------------------------------------
namespace {

struct Blocks {
  double* part = nullptr;
  size_t part_n = 0;
  int tile = 128, splits = 1;
  int* sync = nullptr;
  DevInfo* info = nullptr;
  double* z = nullptr;
  double* diag = nullptr;
};

void carve_blocks(long m, long n, Carver& cv, Blocks& b) {
  syrk_choose((int)m, (int)n, &b.tile, &b.splits);
  b.part_n = syrk_part_elems((int)m, b.tile, b.splits);
  b.part = b.part_n ? cv.take<double>(b.part_n) : nullptr;
  b.sync = cv.take<int>(4 + 2 * cdiv(m, kTB));
  b.diag = cv.take<double>(potrf_diag_elems(m));
  b.info = cv.take<DevInfo>(1);
  b.z = cv.take<double>(m);
}

}  // namespace

extern "C" {

lp_status lp_blocks_workspace_size(int64_t m, int64_t n, size_t* bytes) {
  if (!bytes) return LP_ERR_INVALID_ARG;
  if (m < 1 || n < 1 || m > INT_MAX / 2 || n > INT_MAX / 2) return LP_ERR_SHAPE;
  Carver cv(nullptr);
  Blocks b;
  carve_blocks(m, n, cv, b);
  *bytes = (cv.off + kAlign - 1) / kAlign * kAlign;
  return LP_OK;
}

static lp_status blocks_from(int64_t m, int64_t n, void* ws, size_t ws_bytes, Blocks& b) {
  size_t need = 0;
  lp_status st = lp_blocks_workspace_size(m, n, &need);
  if (st != LP_OK) return st;
  if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) return LP_ERR_WORKSPACE;
  Carver cv(ws);
  carve_blocks(m, n, cv, b);
  return LP_OK;
}

lp_status lp_normal_matrix(int64_t m, int64_t n, const double* A, const double* d, double* M,
                           int64_t ldm, void* workspace, size_t ws_bytes, lp_stream_t stream) {
  if (!A || !d || !M || ldm < m) return LP_ERR_INVALID_ARG;
  Blocks b;
  lp_status st = blocks_from(m, n, workspace, ws_bytes, b);
  if (st != LP_OK) return st;
  launch_syrk_f64(reinterpret_cast<hipStream_t>(stream), (int)m, (int)n, A, n, d, M, ldm, false,
                  b.tile, b.splits, b.part);
  return hip_ok(hipGetLastError());
}

lp_status lp_cholesky(int64_t m, double* M, int64_t ldm, void* workspace, size_t ws_bytes,
                      lp_stream_t stream, int64_t* fail_col, double* min_pivot) {
  if (!M || ldm < m) return LP_ERR_INVALID_ARG;
  Blocks b;
  lp_status st = blocks_from(m, m + 1, workspace, ws_bytes, b);
  if (st != LP_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // a grouped factorization runs part of its updates on a second stream of
  // its own, joined into s before the factorization ends
  CholAux aux;
  hipError_t e = hipSuccess;
  if (chol_grouped((int)m)) {
    e = hipStreamCreateWithFlags(&aux.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&aux.ev_main, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&aux.ev_aux, hipEventDisableTiming);
  }
  DevInfo di;
  if (e == hipSuccess) {
    launch_iter_begin(s, b.info, b.sync, cdiv(m, kTB));
    launch_potrf_f64(s, (int)m, (int)m, M, ldm, b.info, b.diag, &aux);
    e = hipMemcpyAsync(&di, b.info, sizeof(di), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (aux.ev_main) (void)hipEventDestroy(aux.ev_main);
  if (aux.ev_aux) (void)hipEventDestroy(aux.ev_aux);
  if (aux.st) (void)hipStreamDestroy(aux.st);
  if (e != hipSuccess) return LP_ERR_DEVICE;
  const bool broke = di.chol_fail != INT_MAX;
  if (fail_col) *fail_col = broke ? di.chol_fail : -1;
  if (min_pivot) *min_pivot = di.min_pivot;
  return broke ? LP_ERR_BREAKDOWN : LP_OK;
}

lp_status lp_csr_workspace_size(int64_t m, int64_t n, int64_t nnz, size_t* bytes) {
  if (!bytes) return LP_ERR_INVALID_ARG;
  if (m < 1 || n < 1 || m > LP_CSR_MAX_M || !sp_fits(m) || n > INT_MAX / 2 || nnz < 0 ||
      nnz > INT_MAX)
    return LP_ERR_SHAPE;
  Carver cv(nullptr);
  Csc c;
  carve_csc(n, nnz, cv, c);
  *bytes = (cv.off + kAlign - 1) / kAlign * kAlign;
  return LP_OK;
}

lp_status lp_normal_matrix_csr(int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                               const int32_t* col_idx, const double* vals, const double* d,
                               double* M, int64_t ldm, void* workspace, size_t ws_bytes,
                               lp_stream_t stream) {
  size_t need = 0;
  lp_status st = lp_csr_workspace_size(m, n, nnz, &need);
  if (st != LP_OK) return st;
  if (!row_ptr || (nnz > 0 && (!col_idx || !vals)) || !d || !M || ldm < m)
    return LP_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < need || ((uintptr_t)workspace % kAlign) != 0)
    return LP_ERR_WORKSPACE;
  Carver cv(workspace);
  Csc c;
  carve_csc(n, nnz, cv, c);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = csr_prepare(s, m, n, nnz, row_ptr, col_idx, vals, c.flags, c.cp, c.ri, c.cv, c.src, c.map,
                   c.cnt, c.cur);
  if (st != LP_OK) return st;
  launch_sp_syrk(s, m, row_ptr, col_idx, vals, c.cp, c.ri, c.cv, c.map, d, M, ldm);
  return hip_ok(hipGetLastError());
}

lp_status lp_chol_solve(int64_t m, const double* L, int64_t ldm, const double* r, double* dy,
                        void* workspace, size_t ws_bytes, lp_stream_t stream) {
  if (!L || !r || !dy || r == dy || ldm < m) return LP_ERR_INVALID_ARG;
  Blocks b;
  lp_status st = blocks_from(m, m + 1, workspace, ws_bytes, b);
  if (st != LP_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  launch_iter_begin(s, b.info, b.sync, cdiv(m, kTB));
  launch_trsv_fwd(s, (int)m, L, ldm, r, b.z, b.sync, b.info);
  launch_trsv_bwd(s, (int)m, L, ldm, b.z, dy, b.sync, b.info);
  return hip_ok(hipGetLastError());
}

}  // extern "C"
