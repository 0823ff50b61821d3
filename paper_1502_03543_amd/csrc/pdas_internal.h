// Internal declarations shared by the HIP translation units of libpdas.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdas.h"

namespace pdas {

// Per-iteration scalars written by the device and read back by the host.
struct DevInfo {
  double gap_before;
  double gap_after;
  double psi;
  double t;
  double min_pivot;      // bit pattern compared as int64 (positive doubles)
  double refine_resid;
  long long argmax;
  int status;            // lp_status of the step
  int chol_fail;         // first failing pivot column, or INT32_MAX
  int zero_dir;          // 1 when dx = dy = ds = 0 exactly
  int trsv_err;          // a bounded wait in a triangular solve gave up
  int refine_steps;
  int precision_used;
  int lost;              // some updated x_j or s_j <= 0
  int nonfinite;         // psi or a direction component is not finite
  int pad[2];
  // predictor-corrector steps (LP_METHOD_PC)
  double sigma, mu_aff, alpha_aff_p, alpha_aff_d, alpha_p, alpha_d;
};

// Device-side scalar results of input validation.
struct DevCheck {
  int nonfinite;
  int nonpos;
  int pad[2];
};

constexpr int kTB = 64;          // triangular-solve and Cholesky panel block
constexpr int kGemvRows = 64;    // rows per chunk of the transposed GEMV
constexpr int kVecThreads = 256; // threads of the elementwise kernels

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// --- vector kernels (kernels_vec.hip) -------------------------------------
void launch_check_inputs(hipStream_t st, long m, long n, const double* A, const double* b,
                         const double* c, const double* x, const double* y, const double* s,
                         DevCheck* chk);
void launch_fill_i32(hipStream_t st, int* p, int v, long count);
void launch_iter_begin(hipStream_t st, DevInfo* info, int* trsv_sync, int nblk);
// r_d = c - (gy + t g) - s when g != nullptr, else c - gy - s; gy = sum of chunk partials
void launch_dual_resid(hipStream_t st, long m, long n, const double* P, int nchunks,
                       const double* c, const double* s, double* rd);
void launch_prep(hipStream_t st, long n, const double* x, const double* s, const double* rd,
                 double* d, double* w, float* sd = nullptr);
// out = b + sign * A w
void launch_gemv_n(hipStream_t st, long m, long n, const double* A, const double* w,
                   const double* b, double* out, double sign = 1.0);
void launch_gemv_t(hipStream_t st, long m, long n, const double* A, const double* v1,
                   const double* v2, double* P1, double* P2);
int gemv_t_chunks(long m);
void launch_dir(hipStream_t st, long m, long n, const double* P1, const double* P2, int nchunks,
                const double* rd, const double* x, const double* s, const double* d,
                double* dx, double* ds, double* gy, double* g, double* rpart, long long* ipart,
                int* zpart, int* npart);
int dir_blocks(long n);
void launch_step(hipStream_t st, long m, long n, double alpha, int nparts, const double* rpart,
                 const long long* ipart, const int* zpart, const int* npart, const double* dy,
                 const double* x, const double* y, const double* s, const double* dx,
                 const double* ds, const double* g, const double* gy, const double* c,
                 double* xn, double* yn, double* sn, double* rdn, double* gap_part,
                 int* lost_part, DevInfo* info);
int step_blocks(long m, long n);
void launch_finish(hipStream_t st, int nparts, const double* gap_part, const int* lost_part,
                   DevInfo* info);
void launch_gap(hipStream_t st, long n, const double* x, const double* s, double* gap_part,
                double* out);
void launch_copy(hipStream_t st, double* dst, const double* src, long count);
// predictor-corrector (LP_METHOD_PC); amin: 2 * dir_blocks(n) doubles of
// per-block steps to the boundary, mupart: dir_blocks(n) doubles
void launch_pc_aff(hipStream_t st, long n, const double* P1, const double* P2, int nchunks,
                   const double* rd, const double* x, const double* s, const double* d,
                   double* dxa, double* dsa, double* gy, double* amin);
void launch_pc_corr(hipStream_t st, long n, double gap, const double* amin, const double* x,
                    const double* s, const double* rd, const double* d, const double* dxa,
                    const double* dsa, double* mupart, double* q, double* w, DevInfo* info);
void launch_pc_dir(hipStream_t st, long n, const double* P1, int nchunks, const double* rd,
                   const double* x, const double* s, const double* d, const double* q,
                   double* dx, double* ds, double* g, double* amin, int* zpart, int* npart);
void launch_pc_step(hipStream_t st, long m, long n, double eta, const double* amin,
                    const int* zpart, const int* npart, const double* dy, const double* x,
                    const double* y, const double* s, const double* dx, const double* ds,
                    const double* g, const double* gy, const double* c, double* xn, double* yn,
                    double* sn, double* rdn, double* gap_part, int* lost_part, DevInfo* info);
// mixed precision helpers
void launch_to_f32(hipStream_t st, long count, const double* src, float* dst);
void launch_colsq(hipStream_t st, long m, long n, const double* A, double* out);
void launch_scale_partials(hipStream_t st, long n, const double* P, int nchunks, const double* d,
                           double* v);
void launch_axpy(hipStream_t st, long count, const double* x, double* y);
void launch_refine_norms(hipStream_t st, long m, long n, const double* r, const double* dy,
                         const double* d, const double* colsq, double* out);
void launch_lower_f32_to_f64(hipStream_t st, long m, const float* L32, long ld32, double* L64,
                             long ld64);

// --- normal matrix (kernels_syrk.hip) --------------------------------------
// C (row-major lower, ldc) = X diag(w) X^T (w may be null) or, when sub,
// C -= X X^T.  X: mm rows of length K, row stride ldx.  tile 64 or 128:
// split-K over `splits` parts; tile 0: the stream-K kernel (X diag(w) X^T
// only, 16-byte aligned rows and even K; anything else falls back to one
// 64-tile pass).  part: syrk_part_elems(mm, tile, splits) doubles of scratch
// (may be null when that is 0).
void launch_syrk_f64(hipStream_t st, int mm, int K, const double* X, long ldx, const double* w,
                     double* C, long ldc, bool sub, int tile, int splits, double* part,
                     hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);
size_t syrk_part_elems(int mm, int tile, int splits);
void syrk_choose(int mm, int K, int* tile, int* splits);
// FP32: C32 = (X diag(w))(X diag(w))^T (w = sqrt(d), may be null) or C32 -= X X^T.
// Returns false (nothing launched) when K or the rows are not 4-aligned.
bool launch_syrk_f32(hipStream_t st, int mm, int K, const float* X, long ldx, const float* w,
                     float* C, long ldc, bool sub, int splits, float* part,
                     hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);
size_t syrk_part_elems_f32(int mm, int splits);
void syrk_choose_f32(int mm, int K, int* splits);

// --- Cholesky (kernels_chol.hip) -------------------------------------------
// In-place lower Cholesky of M (row-major, ld), m x m; failures recorded in
// info.  diag: scratch for the diagonal blocks, potrf_diag_elems(m) elements.
// The FP64 form factors the first mc columns of an mr-row lower matrix
// (mr >= mc): rows mc .. mr-1 leave as L^-1 applied to them (forward solves
// fused into the factorization).  With mr > mc the trailing updates also
// write the entries (r, c) of those rows for c <= r, so ld must exceed mr - 1.
inline long potrf_diag_elems(long m) { return (long)cdiv(m, kTB) * kTB * kTB; }
// Large factorizations (chol_grouped(mc)) group the panels by four; each
// group's update of the columns beyond the next group then runs on a second
// stream beside the next group's panels when aux is given (both events
// without timing; the factor is the same bit for bit either way).  Without
// aux that update runs in order on st.
struct CholAux {
  hipStream_t st = nullptr;
  hipEvent_t ev_main = nullptr, ev_aux = nullptr;
};
bool chol_grouped(int mc);
// The grouping threshold (columns); lowered only by the CPU emulation of
// the kernels, so that small matrices take the grouped schedule there.
void set_chol_group_min_m(int m);
void launch_potrf_f64(hipStream_t st, int mr, int mc, double* M, long ld, DevInfo* info,
                      double* diag, const CholAux* aux = nullptr);
void launch_potrf_f32(hipStream_t st, int m, float* M, long ld, DevInfo* info, float* diag);

// --- triangular solves (kernels_trsv.hip) ----------------------------------
// z = L^-1 r (fwd) then y = L^-T z (bwd); L row-major lower with ld.
// sync: 2 + 2*nblk ints, zeroed by launch_iter_begin.
void launch_trsv_fwd(hipStream_t st, int m, const double* L, long ld, const double* r, double* z,
                     int* sync, DevInfo* info);
void launch_trsv_bwd(hipStream_t st, int m, const double* L, long ld, const double* z, double* y,
                     int* sync, DevInfo* info);

// --- the paper's Woodbury / Egidi-Maponi solver (kernels_woodbury.hip) ------
constexpr size_t kWoodburyMaxLds = 160 * 1024;  // one workgroup's LDS on gfx950
size_t woodbury_lds_bytes(long m, long n);
bool woodbury_fits(long m, long n);
hipError_t woodbury_prepare();  // allows the kernel its dynamic LDS
void launch_wb_fill(hipStream_t st, long n, double v, double* p);
// Y0 = (L L^T)^-1 A, columns contiguous (Y0[k m + i]); L lower, row-major, ld
void launch_wb_cols(hipStream_t st, int m, int n, const double* L, long ld, const double* A,
                    double* Y0);
// dy = (A D A^T)^-1 rhs from x0 = (A A^T)^-1 rhs by the rank-one recurrence
void launch_woodbury(hipStream_t st, int m, int n, const double* A, const double* d,
                     const double* Y0, const double* x0, double* dy, DevInfo* info);

// --- sparse A in canonical CSR (kernels_sparse.hip) ------------------------
constexpr size_t kSparseMaxLds = 160 * 1024;
size_t sp_syrk_lds_bytes(long m);
bool sp_fits(long m);               // the normal-matrix kernel's LDS row fits
hipError_t sp_prepare();            // allows that kernel its dynamic LDS
// flags: bit 0 bad structure, bit 1 non-finite value (caller zeroes them)
void launch_sp_check(hipStream_t st, long m, long n, long nnz, const int64_t* rp, const int* ci,
                     const double* v, int* flags);
// CSC of a checked CSR: cp (n + 1), ri / cv / src (nnz), map (nnz: CSC
// position of each CSR entry); cnt, cur: n ints of scratch
void launch_sp_transpose(hipStream_t st, long m, long n, long nnz, const int64_t* rp,
                         const int* ci, const double* v, int* cnt, int* cur, int64_t* cp,
                         int* ri, double* cv, int* src, int* map);
// out = base + sign * A w
void launch_sp_gemv_n(hipStream_t st, long m, long nnz, const int64_t* rp, const int* ci,
                      const double* v, const double* w, const double* base, double* out,
                      double sign = 1.0);
// g1 = A^T v1 and, when v2, g2 = A^T v2 (full sums: one chunk)
void launch_sp_gemv_t(hipStream_t st, long n, long nnz, const int64_t* cp, const int* ri,
                      const double* cv, const double* v1, const double* v2, double* g1,
                      double* g2);
// lower triangle of M = A diag(d) A^T (row-major, ldm)
void launch_sp_syrk(hipStream_t st, long m, const int64_t* rp, const int* ci, const double* v,
                    const int64_t* cp, const int* ri, const double* cv, const int* map,
                    const double* d, double* M, long ldm);

// --- reverse mode (kernels_adjoint.hip) -------------------------------------
void launch_zero(hipStream_t st, double* p, long count);
void launch_adj_tbar(hipStream_t st, long m, long n, const double* xb, const double* dx,
                     const double* sb, const double* ds, const double* yb, const double* dy,
                     double* part, double* out);
void launch_adj_a(hipStream_t st, long m, long n, double alpha, const DevInfo* info,
                  const double* tbar, const double* x, const double* s, const double* d,
                  const double* dx, const double* ds, double* xb, double* sb, const double* yb,
                  double* dsb, double* db, double* dyb);
void launch_adj_b(hipStream_t st, long m, long n, const double* P, int nchunks, const double* g,
                  const double* rd, const double* d, const double* x, const double* s,
                  const double* lam, const double* dsb, double* db, double* xb, double* sb,
                  double* cb, double* rdb, double* bb, double* v1, double* v2, double* v3);
void launch_rank3(hipStream_t st, long m, long n, double* Ab, const double* u1, const double* v1,
                  const double* u2, const double* v2, const double* u3, const double* v3);

// --- batched solver (kernels_batch.hip) ------------------------------------
struct BatchLP {
  int m, n, ldm, pad;
  long a_off;     // element offset of A_i in the packed matrices
  long vm, vn;    // element offsets of the m- and n-vectors of LP i
  long M_off;     // element offset of M_i (ldm x m) in the matrix pool
  long tape_off;  // element offset of LP i's tape
  long diag_off;  // element offset of LP i's diagonal-block scratch
  // mixed precision (FP32 factor): rows of A32 and sqrt(d) padded to n4 =
  // n rounded up to 4 with zeros; M32 is ld32 x m, ld32 = m rounded up to 4
  long a32_off;   // element offset of A32_i in the FP32 matrix pool
  long m32_off;   // element offset of M32_i
  long vn4;       // element offset of LP i's padded n-vectors (sqrt(d) in FP32)
  int ld32, n4;
};

struct BatchState {
  int status;     // lp_status; LP_OK while active
  int iters;      // directions taken
  int cur;        // which iterate buffer holds the current iterate
  int pad;
  double gap;     // x^T s of the current iterate
  double last_psi, last_t;
  long long last_argmax;
};

struct BatchArgs {
  int count;
  int max_iter;
  double alpha, tol;
  const BatchLP* lps;
  BatchState* state;
  const double* A;      // caller's packed matrices (offsets a_off)
  const double* b;      // workspace copies, packed by vm / vn
  const double* c;
  double* x[2];
  double* y[2];
  double* s[2];
  double* rd[2];
  double *d, *w, *g, *gy, *dx, *ds, *rhs, *z, *dy, *M;
  double* diag;         // diagonal blocks of the factors (potrf_diag_elems(m) per LP)
  double* tape;
  int tape_cap;
  int* active;          // LPs still iterating after the last step
  int* go;              // per LP: 1 when it takes (or reverses) a step in this launch sequence
  int* fail;            // per LP: first failing Cholesky pivot column, INT_MAX for none
  unsigned long long* minp;  // per LP: smallest pivot (bit pattern of a positive double)
  double* psi;          // per LP: psi of the current direction
  long long* arg;       // per LP: its first maximiser (x block j, s block n + j)
  int tile;             // edge of the normal-matrix tiles (32, 64, 128; updates: 32, 64)
  int nslice;           // 256-column slices of the widest LP
  double* dpv;          // per LP and slice: the slice's ratio-test maximum,
  long long* dpi;       //   its first maximiser
  int* dpf;             //   and flags (1 nonzero direction, 2 non-finite ratio)
  // mixed precision (lp_options.precision == LP_PREC_MIXED; null otherwise)
  int mixed;
  double refine_tol, switch_gap;
  int refine_max;
  float* A32;           // FP32 copies of the A_i (padded rows)
  float *M32, *diag32, *sd32;
  double *r, *delta, *v;  // refinement residual, correction, d o (A^T dy)
  int* fp32_mode;       // per LP: FP32 factor still allowed (cleared for good)
  int* m32;             // per LP: FP32 factor tried in this iteration
  int* go64;            // per LP: FP64 factor in this iteration
  int* refm;            // per LP: refinement still running
  int* ref_status;      // per LP: 0 running, 1 converged, 2 failed, 3 none
  int* ref_steps;       // per LP: corrections taken in this iteration
  double* ref_prev;     // per LP: previous correction's max norm
};

// Adjoint pools of a batch (packed like the forward vectors; Abar like A).
struct BatchAdj {
  double *xb, *yb, *sb, *dsb, *db, *dyb, *lam, *h, *rdb, *bbar, *cbar;
  double* Abar;  // caller's output, may be null
  int* err;
  // Abar's rank-3 terms of every reverse step k, formed once after the sweep:
  // ufac[(3 k + r) sm + vm + i] and vfac[(3 k + r) sn + vn + j], r = 0..2
  double *ufac, *vfac;
  long sm, sn;
  int max_n;  // largest n of the batch (grid of the column-wise launch)
};

// One forward iteration of every active LP (k < 0), or the recomputation
// and reverse of step k (k >= 0, with adj), as a fixed sequence of launches
// whose shapes depend only on count and max_m (so it can be captured once).
void launch_batch_step(hipStream_t st, const BatchArgs& args, int max_m, int k,
                       const BatchAdj* adj);
// Abar of every LP from the factors the reverse sweep stored (steps taken
// by that LP, capped at tape_cap), in 64 x 64 tiles (max_tiles per LP).
void launch_babar(hipStream_t st, int count, int max_tiles, const BatchLP* lps,
                  const BatchState* state, const BatchAdj& adj, int tape_cap, double* Abar);
void launch_batch_setup(hipStream_t st, int count, const BatchLP* lps, BatchState* state,
                        const double* Ap, const double* c, const double* x, const double* y,
                        const double* s, double* rd);
// batched building blocks (kernels_syrk.hip, kernels_chol.hip)
// mixed precision of the batch (kernels_batch_mixed.hip): the FP32 copies
// of A (setup), then per iteration the FP32 factor of the LPs that try it,
// up to refine_max FP64 corrections, and the FP64 factor for the others
void launch_bmix_setup(hipStream_t st, int count, int max_m, const BatchLP* lps, const double* A,
                       float* A32);
void launch_bmix_factor(hipStream_t st, const BatchArgs& a, int max_m);
void launch_bsyrk_normal_f32(hipStream_t st, int count, int max_m, int tile, const BatchLP* lps,
                             const int* go, const float* A32, const float* sd32, float* M32);
void launch_bsyrk_trailing_f32(hipStream_t st, int count, int max_m, int tile,
                               const BatchLP* lps, const int* go, float* M32, int p);
void launch_bpotrf_panel_f32(hipStream_t st, int count, int max_m, const BatchLP* lps,
                             const int* go, float* M32, float* diag32, int p, int* fail,
                             unsigned long long* minp_bits);
void launch_bdiag_to_m_f32(hipStream_t st, int count, int max_m, const BatchLP* lps,
                           const int* go, float* M32, const float* diag32);
// tile: 32, 64 or 128 (the edge of the lower tiles).  With rhs given, the
// 32- and 64-tile kernels also form rhs_i = b_i + A_i w_i and the call
// returns true; otherwise (and always for 128) rhs is the caller's to form.
bool launch_bsyrk_normal(hipStream_t st, int count, int max_m, int tile, const BatchLP* lps,
                         const int* go, const double* A, const double* d, double* Mpool,
                         const double* w, const double* b, double* rhs);
void launch_bsyrk_trailing(hipStream_t st, int count, int max_m, int tile, const BatchLP* lps,
                           const int* go, double* Mpool, int p);
void launch_bpotrf_panel(hipStream_t st, int count, int max_m, const BatchLP* lps, const int* go,
                         double* Mpool, double* diagpool, int p, int* fail,
                         unsigned long long* minp_bits);
void launch_bdiag_to_m(hipStream_t st, int count, int max_m, const BatchLP* lps, const int* go,
                       double* Mpool, const double* diagpool);

}  // namespace pdas
