/*
 * pdas.h -- C ABI of the MI355X (gfx950) Primal-Dual Affine Scaling library.
 *
 * Problem (Section 1, equations (primal) and (dual) of Divakar, "Primal Dual
 * Affine Scaling on GPUs", arXiv 1502.03543):
 *     minimise c^T x  s.t.  A x = b, x >= 0        (primal)
 *     maximise b^T y  s.t.  A^T y + s = c, s >= 0  (dual)
 * with A in R^{m x n}, full row rank, m < n.
 *
 * Each iteration follows the Section 3 algorithm: solve the Newton system
 * (bigsystem) for (dx, dy, ds), take the ratio test
 *     psi = max{ max_j(-dx_j/x_j), max_j(-ds_j/s_j) },
 * set alpha := 1 when psi == 1, step (x, y, s) += (alpha/psi)(dx, dy, ds),
 * and stop as optimal after a psi == 1 step.  The Newton system is reduced as
 * in Section 5 (equation (bigsystem2) and the formulas below it) to the normal
 * equations (A D A^T) dy = rhs with D = diag(x/s), written with residuals:
 *     r_d = c - A^T y - s,  rhs = b + A (d o r_d),
 *     ds  = r_d - A^T dy,   dx  = -x - d o ds,
 * which on a feasible iterate is the paper's (ADA^T) dy = Ax, ds = -A^T dy,
 * dx = D(-ds) - x.  A D A^T is factored by Cholesky (Section 5.1).
 *
 * Conventions for every entry point:
 *  - Matrices are row-major; A is m x n with leading dimension n.
 *  - Pointers documented "device" are HIP device (or managed) memory.
 *    Pointers documented "host" are ordinary host memory.
 *  - The library never allocates device memory.  The caller supplies one
 *    device workspace, sized by lp_workspace_size / lp_batch_workspace_size,
 *    that the library carves up.  Handles themselves are small host objects.
 *  - All device work is ordered on the stream given to lp_setup.  Functions
 *    that return host values (info, results) synchronise that stream.  A
 *    handle with m >= 4096 also owns a second stream (default priority) and
 *    two events: part of each factorization's trailing update runs there,
 *    and the caller's stream waits for it before the factorization ends, so
 *    the ordering seen by the caller is unchanged.  lp_destroy releases them.
 *  - One handle must not be used from two host threads at once.
 *  - Nothing throws or aborts across this ABI: every function returns an
 *    lp_status; on an error the handle keeps its last valid iterate.
 */
#ifndef PDAS_H
#define PDAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same type as HIP's hipStream_t; NULL is the default stream. */
typedef struct ihipStream_t* lp_stream_t;

typedef enum lp_status {
  LP_OK = 0,               /* call succeeded; for lp_iterate: loop continues  */
  LP_CONVERGED = 1,        /* x^T s < gap_tol before the next direction      */
  LP_OPTIMAL_PSI1 = 2,     /* psi == 1: full step taken, iterate optimal (Section 3) */
  LP_OPTIMAL_ZERO_DIR = 3, /* dx = dy = ds = 0 exactly (Section 3)           */
  LP_MAX_ITER = 4,         /* iteration limit reached                        */
  LP_ERR_INVALID_ARG = -1, /* NULL pointer, non-finite data, alpha not in (0,1) ... */
  LP_ERR_SHAPE = -2,       /* m < 1 or m >= n (Section 1 assumes m < n)       */
  LP_ERR_NOT_INTERIOR = -3,/* some x0_j <= 0 or s0_j <= 0                    */
  LP_ERR_BREAKDOWN = -4,   /* Cholesky met a pivot that is not finite and > 0 */
  LP_ERR_NONPOS_PSI = -5,  /* psi not finite or <= 0                          */
  LP_ERR_LOST_INTERIOR = -6,/* a step left some x_j or s_j <= 0 (step undone) */
  LP_ERR_WORKSPACE = -7,   /* workspace NULL, too small or misaligned (256 B) */
  LP_ERR_NO_TAPE = -8,     /* lp_backward without a recorded tape             */
  LP_ERR_DEVICE = -9       /* a HIP runtime call failed                       */
} lp_status;

typedef enum lp_precision {
  LP_PREC_FP64 = 0,  /* every step in FP64                                     */
  LP_PREC_MIXED = 1  /* FP32 normal matrix and factor with FP64 refinement,
                        switching to FP64 for good (see lp_options)            */
} lp_precision;

typedef enum lp_method {
  LP_METHOD_AFFINE = 0, /* the Section 3 algorithm (primal-dual affine scaling) */
  LP_METHOD_PC = 1      /* Mehrotra's predictor-corrector, which Section 4
                           (previous work) cites: the Section 3 direction as
                           predictor, sigma = (mu_aff/mu)^3 from its steps to
                           the boundary, a corrector solve with the same factor
                           and third right-hand side -Xs - dX_aff dS_aff e +
                           sigma mu e, then primal and dual steps of
                           min(1, alpha * step to the boundary).  FP64 only, no
                           tape (LP_ERR_INVALID_ARG otherwise); not for batches */
} lp_method;

typedef enum lp_solver {
  LP_SOLVER_CHOLESKY = 0, /* normal matrix on the matrix cores, blocked Cholesky,
                             triangular solves (Section 5.1's usual method)     */
  LP_SOLVER_WOODBURY = 1  /* the paper's Section 5 solver: A D A^T split as
                             A A^T plus the rank-one terms (d_l - 1) a_l a_l^T,
                             applied by the Egidi-Maponi recurrence to
                             (A A^T)^-1 [A | rhs] (factor of A A^T and
                             (A A^T)^-1 A formed once at lp_setup).  The n terms
                             run in one workgroup with Y in LDS, so it needs
                             8 ((n + 1) ld + n + 16 m) <= 160 KiB, ld = m rounded up
                             to odd (LP_ERR_SHAPE otherwise: e.g. m = 64,
                             n = 256 fits); FP64, LP_METHOD_AFFINE, no tape
                             (LP_ERR_INVALID_ARG otherwise).  A rank-deficient
                             A makes lp_setup return LP_ERR_BREAKDOWN; a
                             recurrence denominator that is not a finite
                             positive number ends the run with it, and
                             min_pivot reports the smallest denominator      */
} lp_solver;

typedef struct lp_options {
  double alpha;            /* step fraction, 0 < alpha < 1 (Section 3)          */
  int32_t precision;       /* lp_precision                                       */
  int32_t tape_capacity;   /* iterations whose start iterate is recorded for
                              lp_backward (0: no tape)                           */
  double mixed_switch_gap; /* MIXED: use FP64 once x^T s < this (default 1e-6)   */
  double refine_tol;       /* MIXED: refinement succeeds when the relative
                              correction ||delta_i||/||dy|| (or, once the
                              corrections contract by q < 1/2, the remaining
                              error estimate ||delta_i|| q/(1-q) / ||dy||) is
                              <= refine_tol (default 2^-46 ~ 1.4e-14)            */
  int32_t refine_max;      /* MIXED: corrections before falling back to FP64; a
                              correction that does not halve the previous one,
                              or an FP32 pivot that is not positive, also falls
                              back (default 5)                                   */
  int32_t profile;         /* 2: time only the normal-matrix kernel with HIP
                              events on the handle's stream (two events per
                              iteration); any other non-zero value: time
                              every phase (see lp_get_timings)                    */
  int32_t syrk_tile;       /* FP64 normal-matrix kernel: 0 (library's choice:
                              the stream-K kernel, 128 x 128 tiles and one
                              equal share of the work per compute unit, when
                              m >= 512 and n >= 1024; split-K otherwise), or
                              the split-K kernel with 64 or 128 tiles; see
                              paper_1502_03543_amd/autotune.py                   */
  int32_t syrk_splits;     /* FP64 split-K parts of the sum over j: 0 (library's
                              choice) or 1..64; non-zero selects split-K (with
                              128 tiles unless syrk_tile says 64)                */
  int32_t syrk32_splits;   /* FP32 normal-matrix split (MIXED): 0 or 1..64      */
  int32_t method;          /* lp_method (default LP_METHOD_AFFINE)               */
  int32_t solver;          /* lp_solver (default LP_SOLVER_CHOLESKY)             */
  int32_t batch_tile;      /* lp_batch_*: normal-matrix and trailing-update tile
                              edge, 0 (library's choice: FP64 normal matrix
                              on 64-edge tiles for LPs with m > 128 and
                              32-edge tiles for the others, trailing updates
                              on 32, the FP32 path on 64), 32, 64 or 128
                              (128: FP64 normal matrix on 128 x 128 tiles of
                              eight wavefronts; trailing updates and the FP32
                              normal matrix then use 64); see
                              paper_1502_03543_amd/autotune.py.  Ignored by the
                              single-LP calls (which accept only these values) */
  int32_t batch_graph_iters; /* lp_batch_solve: iterations captured per
                              hipGraph and replayed between host checks, 0
                              (library's choice: 4) or 1..16                    */
  int32_t reserved;        /* must be 0                                          */
  int32_t reserved2;       /* must be 0                                          */
} lp_options;

/* Fill *opt with the defaults: alpha 0.95, FP64, no tape, switch gap 1e-6,
 * refine_tol 2^-46, refine_max 5, no profiling, library tile choices. */
void lp_options_default(lp_options* opt);

typedef struct lp_iter_info {
  int32_t k;              /* index of the direction just taken (0-based)       */
  int32_t status;         /* lp_status of the step (LP_OK while continuing)    */
  double gap_before;      /* x^T s before the step                             */
  double gap_after;       /* x^T s after the step                              */
  double psi;             /* ratio-test value (NaN for LP_METHOD_PC)           */
  double t;               /* step length alpha_eff / psi                       */
  int64_t argmax;         /* j in [0,n): x-block; n + j: s-block                */
  double min_pivot;       /* smallest Cholesky pivot (squared diagonal of L)    */
  int32_t precision_used; /* lp_precision of this step's factor                */
  int32_t refine_steps;   /* refinement steps taken (MIXED)                    */
  double refine_resid;    /* estimated relative error of dy after refinement   */
  double alpha_primal;    /* step applied to x (LP_METHOD_AFFINE: t)           */
  double alpha_dual;      /* step applied to y and s (LP_METHOD_AFFINE: t)     */
  double sigma;           /* centring parameter (LP_METHOD_PC; 0 otherwise)    */
} lp_iter_info;

typedef struct lp_result {
  int32_t status;         /* terminal lp_status                                 */
  int32_t iters;          /* directions taken                                   */
  double gap;             /* x^T s of the final iterate                         */
  double primal_obj;      /* c^T x                                              */
  double dual_obj;        /* b^T y                                              */
} lp_result;

/* Accumulated device time per phase (milliseconds, HIP events on the
 * handle's stream) over the iterations run with lp_options.profile set. */
typedef struct lp_timings {
  double normal_kernel_ms; /* the normal-matrix MFMA kernel alone             */
  double normal_ms;        /* normal matrix including the split-K reduction    */
  double potrf_ms;         /* blocked Cholesky                                 */
  double trsv_ms;          /* both triangular solves                           */
  double other_ms;         /* GEMVs, direction, ratio test, step, refinement   */
  double iter_ms;          /* whole iterations                                 */
  int64_t iterations;      /* iterations timed                                 */
  int64_t normal_launches; /* normal-matrix kernel launches timed              */
} lp_timings;

typedef struct lp_handle lp_handle;

/* Human-readable name of a status ("LP_CONVERGED", ...). Never NULL. */
const char* lp_status_string(int32_t status);

/* Bytes of device workspace lp_setup needs for an m x n problem with the given
 * options (opt NULL: defaults).  Errors: LP_ERR_SHAPE, LP_ERR_INVALID_ARG. */
lp_status lp_workspace_size(int64_t m, int64_t n, const lp_options* opt, size_t* bytes);

/* Create a handle for one LP.  A (device, m x n row-major) is borrowed and must
 * stay valid and unchanged for the handle's lifetime.  b (m), c (n), x0 (n),
 * y0 (m), s0 (n) are device vectors copied into the workspace.  workspace is a
 * device buffer of at least lp_workspace_size bytes, 256-byte aligned, owned
 * by the caller and used exclusively by this handle until lp_destroy.
 * Validates: shape (LP_ERR_SHAPE), finiteness and alpha (LP_ERR_INVALID_ARG),
 * x0 > 0 and s0 > 0 (LP_ERR_NOT_INTERIOR).  Synchronises the stream.
 * On error *h is set to NULL. */
lp_status lp_setup(lp_handle** h, int64_t m, int64_t n, const double* A, const double* b,
                   const double* c, const double* x0, const double* y0, const double* s0,
                   const lp_options* opt, void* workspace, size_t ws_bytes,
                   lp_stream_t stream);

/* Sparse A (Section 7 names sparse systems as the method's next step, with
 * coalesced access as the difficulty).  A is given in canonical CSR: row_ptr
 * (device, m + 1 int64: row_ptr[0] = 0, non-decreasing, row_ptr[m] = nnz),
 * col_idx (device, nnz int32, strictly increasing within each row: sorted,
 * no duplicates, in [0, n)), vals (device, nnz doubles, finite).  The three
 * arrays are borrowed like A in lp_setup.  The library builds the transpose
 * (CSC) once in the workspace; the products A w and A^T v then run on the
 * CSR and the CSC, the normal matrix A D A^T on both (its dense lower
 * triangle: the Cholesky, the triangular solves and every vector kernel are
 * those of the dense path, and so are the results up to the rounding order
 * of the sums).  Supported: FP64, LP_SOLVER_CHOLESKY, LP_METHOD_AFFINE and
 * LP_METHOD_PC, no tape; other options give LP_ERR_INVALID_ARG.  The
 * normal-matrix kernel keeps one row of M in LDS, so m <= LP_CSR_MAX_M
 * (LP_ERR_SHAPE above).  nnz = 0 is accepted (the first iteration then
 * reports LP_ERR_BREAKDOWN). */
#define LP_CSR_MAX_M 16384

/* Workspace bytes for lp_setup_csr.  Errors: LP_ERR_SHAPE (as lp_workspace_size,
 * m > LP_CSR_MAX_M, nnz < 0 or nnz > INT32_MAX), LP_ERR_INVALID_ARG. */
lp_status lp_workspace_size_csr(int64_t m, int64_t n, int64_t nnz, const lp_options* opt,
                                size_t* bytes);

/* lp_setup for a CSR matrix A.  Validates on the device what lp_setup does,
 * and the CSR structure and values (LP_ERR_INVALID_ARG when they break the
 * rules above).  The returned handle takes lp_iterate, lp_solve,
 * lp_get_iterate, lp_get_direction, lp_get_timings and lp_destroy;
 * lp_backward returns LP_ERR_NO_TAPE.  Synchronises the stream. */
lp_status lp_setup_csr(lp_handle** h, int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                       const int32_t* col_idx, const double* vals, const double* b,
                       const double* c, const double* x0, const double* y0, const double* s0,
                       const lp_options* opt, void* workspace, size_t ws_bytes,
                       lp_stream_t stream);

/* One pass of the Section 3 loop body: direction, zero-direction test, ratio
 * test, psi == 1 rule, step.  Returns LP_OK to continue, LP_OPTIMAL_PSI1,
 * LP_OPTIMAL_ZERO_DIR or an error.  info (host, nullable) receives the
 * step's values; the call synchronises the stream. */
lp_status lp_iterate(lp_handle* h, lp_iter_info* info);

/* The Section 3 loop: before each direction stop with LP_CONVERGED when
 * x^T s < gap_tol, or with LP_MAX_ITER after max_iter directions from this
 * call.  result (host, nullable) receives the summary.  log (host, nullable,
 * max_iter entries) receives one entry per direction taken. */
lp_status lp_solve(lp_handle* h, double gap_tol, int32_t max_iter, lp_result* result,
                   lp_iter_info* log);

/* Copy the current iterate to device buffers x (n), y (m), s (n); any may be
 * NULL.  Stream-ordered, does not synchronise. */
lp_status lp_get_iterate(const lp_handle* h, double* x, double* y, double* s);

/* Copy the direction (dx, dy, ds) of the most recent lp_iterate to device
 * buffers dx (n), dy (m), ds (n); any may be NULL.  Stream-ordered. */
lp_status lp_get_direction(const lp_handle* h, double* dx, double* dy, double* ds);

/* Copy the accumulated phase timings (zero when profiling is off). */
lp_status lp_get_timings(const lp_handle* h, lp_timings* out);

/* Reverse mode through the directions taken since lp_setup, for a scalar loss
 * on the final iterate.  Needs lp_options.tape_capacity >= that number of
 * directions (LP_ERR_NO_TAPE otherwise).  Inputs: xbar_K (device, n; required),
 * ybar_K (m) and sbar_K (n) (device, nullable: zero) are the loss gradients
 * with respect to the final x, y, s.  Outputs (device, each nullable): Abar
 * (m x n row-major), bbar (m), cbar (n), x0bar (n), y0bar (m), s0bar (n), the
 * gradients with respect to the inputs of lp_setup.  Each recorded step is
 * recomputed in FP64 from its start iterate and dual residual (normal matrix
 * and Cholesky factor included; bit-identical to an FP64 forward pass), and
 * the factor serves the solve with the symmetric M.  A psi == 1 step length
 * is treated as constant.  Uses the handle's workspace and stream and leaves
 * its iterate unchanged; synchronises. */
lp_status lp_backward(lp_handle* h, const double* xbar_K, const double* ybar_K,
                      const double* sbar_K, double* Abar, double* bbar, double* cbar,
                      double* x0bar, double* y0bar, double* s0bar);

/* Copy the start iterate of recorded step k (0 <= k < directions recorded)
 * to device buffers x (n), y (m), s (n); any may be NULL.  LP_ERR_NO_TAPE
 * without a tape or for k out of range.  Stream-ordered. */
lp_status lp_tape_row(const lp_handle* h, int32_t k, double* x, double* y, double* s);

/* Release the handle (host memory only; the workspace stays the caller's). */
lp_status lp_destroy(lp_handle* h);

/* ------------------------------------------------------------------------- */
/* Batched solver: count independent LPs of individual shapes (m_i, n_i), each  */
/* running the same Section 3 iteration.  One iteration of the whole batch is  */
/* a fixed sequence of launches (normal-matrix tiles, Cholesky panels and      */
/* trailing updates of every LP at once, per-LP direction and step); several   */
/* iterations are captured into one hipGraph and replayed.  LPs that stopped   */
/* skip every launch.  FP64, or mixed precision per LP (below).              */
/* ------------------------------------------------------------------------- */
typedef struct lp_batch lp_batch;

/* Workspace bytes for a batch; m, n are host arrays of length count, each LP
 * needing 1 <= m_i < n_i (LP_ERR_SHAPE otherwise).  Options: LP_METHOD_AFFINE
 * and LP_SOLVER_CHOLESKY; precision LP_PREC_FP64 or LP_PREC_MIXED.  MIXED
 * runs the single-LP mixed scheme per LP inside the captured iteration: an
 * FP32 normal matrix and factor, up to refine_max (<= 16) FP64 corrections,
 * and for an LP whose FP32 pivot fails, whose corrections stall or that does
 * not converge, the FP64 factor in the same iteration and from then on (also
 * once its gap is below mixed_switch_gap); no tape with MIXED.
 * lp_batch_iterate reports per LP the factor used (precision_used) and the
 * corrections taken.  Other options give LP_ERR_INVALID_ARG. */
lp_status lp_batch_workspace_size(int32_t count, const int64_t* m, const int64_t* n,
                                  const lp_options* opt, size_t* bytes);

/* A_packed (device) holds the matrices back to back: LP i row-major m_i x n_i
 * starting at element a_off[i] (host array); it is borrowed for the handle's
 * lifetime.  b and y0 (device) hold LP i's m-vector at element v_off_m[i],
 * c, x0 and s0 (device) its n-vectors at v_off_n[i] (host arrays); they are
 * copied.  Validation as lp_setup for every LP; any failure fails the call
 * (first error by LP index: LP_ERR_INVALID_ARG before LP_ERR_NOT_INTERIOR).
 * Synchronises the stream. */
lp_status lp_batch_setup(lp_batch** h, int32_t count, const int64_t* m, const int64_t* n,
                         const double* A_packed, const int64_t* a_off, const double* b,
                         const double* c, const double* x0, const double* y0,
                         const double* s0, const int64_t* v_off_m, const int64_t* v_off_n,
                         const lp_options* opt, void* workspace, size_t ws_bytes,
                         lp_stream_t stream);

/* Run the batch until every LP has stopped: x^T s < gap_tol before a
 * direction (LP_CONVERGED), psi == 1 (LP_OPTIMAL_PSI1), an error, or max_iter
 * directions in total since setup (LP_MAX_ITER).  status and iters (host,
 * count entries each, nullable) receive the per-LP outcome; *n_converged
 * (nullable) counts LP_CONVERGED and LP_OPTIMAL_PSI1.  Returns LP_OK unless a
 * HIP call failed. */
lp_status lp_batch_solve(lp_batch* h, double gap_tol, int32_t max_iter, int32_t* status,
                         int32_t* iters, int32_t* n_converged);

/* One pass of the Section 3 loop body for every LP of the batch that is still
 * running, as one iteration of lp_batch_solve: an LP whose x^T s < gap_tol
 * stops first with LP_CONVERGED (gap_tol 0: no gap test); every other running
 * LP takes one direction, the zero-direction test, the ratio test, the
 * psi == 1 rule and the step.  There is no iteration limit here; LPs stopped
 * earlier (by this call or lp_batch_solve) are left as they are.
 * status (host, count entries, nullable) receives each LP's status after the
 * call (LP_OK while it keeps running).  info (host, count entries, nullable)
 * receives, per LP in the caller's order: k, the index of the direction
 * computed in this call, or -1 when the LP took none (then only status and
 * gap_before = gap_after, its current x^T s, are meaningful); status;
 * gap_before and gap_after; psi (NaN after a breakdown); t and argmax (of the
 * step taken, or undone for LP_ERR_LOST_INTERIOR; 0 and -1 otherwise);
 * min_pivot (the smallest Cholesky pivot of the step); precision_used
 * (LP_PREC_FP64).  Returns LP_OK unless a HIP call failed
 * (LP_ERR_DEVICE) or h is NULL or gap_tol is negative or NaN
 * (LP_ERR_INVALID_ARG).  Synchronises. */
lp_status lp_batch_iterate(lp_batch* h, double gap_tol, int32_t* status, lp_iter_info* info);

/* Copy the current iterates to device buffers x (sum n_i), y (sum m_i) and
 * s (sum n_i), packed contiguously in LP order (LP i's n-vector starts at
 * n_0 + ... + n_{i-1}); any may be NULL.  Stream-ordered. */
lp_status lp_batch_get_iterate(const lp_batch* h, double* x, double* y, double* s);

/* Reverse mode of the batch through the directions each LP took since
 * lp_batch_setup (needs lp_options.tape_capacity >= the largest count;
 * LP_ERR_NO_TAPE otherwise), for a scalar loss on the final iterates.  xbar_K
 * (required), ybar_K, sbar_K (nullable: zero) are packed like
 * lp_batch_get_iterate's outputs; Abar (nullable) is packed like A_packed
 * (offsets a_off); bbar, cbar, x0bar, y0bar, s0bar (nullable) are packed like
 * the iterates.  Every recorded step is recomputed from its start iterate and
 * dual residual in FP64 and its Cholesky factor serves the solve with M; the
 * steps' rank-3 terms of Abar are kept in the workspace and summed once after
 * the sweep.  Synchronises. */
lp_status lp_batch_backward(lp_batch* h, const double* xbar_K, const double* ybar_K,
                            const double* sbar_K, double* Abar, double* bbar, double* cbar,
                            double* x0bar, double* y0bar, double* s0bar);

/* Start iterates of recorded step k of every LP, packed like
 * lp_batch_get_iterate (LPs that took fewer than k + 1 steps are left
 * untouched).  LP_ERR_NO_TAPE without a tape or for k >= tape_capacity. */
lp_status lp_batch_tape_row(const lp_batch* h, int32_t k, double* x, double* y, double* s);

/* Release the batch handle (host memory only). */
lp_status lp_batch_destroy(lp_batch* h);

/* ------------------------------------------------------------------------- */
/* Building blocks of one iteration, exposed for callers that drive their own  */
/* loop (and for kernel-level checks).  Same conventions as above; scratch     */
/* comes from a caller workspace of lp_blocks_workspace_size bytes.            */
/* ------------------------------------------------------------------------- */

/* Workspace bytes for lp_normal_matrix / lp_cholesky / lp_chol_solve on an
 * m x n problem. */
lp_status lp_blocks_workspace_size(int64_t m, int64_t n, size_t* bytes);

/* Normal matrix of the Section 5 reduced system: M = A diag(d) A^T, written to
 * the lower triangle (i >= j) of M (device, row-major, leading dimension
 * ldm >= m); the strict upper triangle is left untouched.  A (device, m x n
 * row-major), d (device, n).  Stream-ordered, does not synchronise. */
lp_status lp_normal_matrix(int64_t m, int64_t n, const double* A, const double* d, double* M,
                           int64_t ldm, void* workspace, size_t ws_bytes, lp_stream_t stream);

/* In-place Cholesky M = L L^T (Section 5.1) of the lower triangle of M
 * (device, row-major, ldm).  For m >= 4096 the call creates a second stream
 * and two events for the duration of the factorization (LP_ERR_DEVICE if
 * that fails).  Synchronises; *fail_col (host, nullable)
 * receives -1, or the first column whose pivot is not a finite positive
 * number (then LP_ERR_BREAKDOWN is returned and M holds partial results);
 * *min_pivot (host, nullable) the smallest accepted pivot. */
lp_status lp_cholesky(int64_t m, double* M, int64_t ldm, void* workspace, size_t ws_bytes,
                      lp_stream_t stream, int64_t* fail_col, double* min_pivot);

/* dy = L^-T L^-1 r for the factor left by lp_cholesky; r, dy device m-vectors
 * (may not alias).  Stream-ordered, does not synchronise. */
lp_status lp_chol_solve(int64_t m, const double* L, int64_t ldm, const double* r, double* dy,
                        void* workspace, size_t ws_bytes, lp_stream_t stream);

/* Workspace bytes for lp_normal_matrix_csr (the CSC of A and its index maps). */
lp_status lp_csr_workspace_size(int64_t m, int64_t n, int64_t nnz, size_t* bytes);

/* lp_normal_matrix for A in canonical CSR (rules as lp_setup_csr): M = A
 * diag(d) A^T written to the lower triangle (i >= j) of M (device,
 * row-major, ldm >= m), with the kernel lp_setup_csr's handle uses.
 * Checks the CSR on the device and builds its transpose in the workspace on
 * every call (LP_ERR_INVALID_ARG for a bad structure or value), so it
 * synchronises.  Errors: LP_ERR_SHAPE (m < 1, n < 1, m > LP_CSR_MAX_M, nnz
 * out of range), LP_ERR_WORKSPACE, LP_ERR_DEVICE. */
lp_status lp_normal_matrix_csr(int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                               const int32_t* col_idx, const double* vals, const double* d,
                               double* M, int64_t ldm, void* workspace, size_t ws_bytes,
                               lp_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Allocation-free entry point                                                 */
/* ------------------------------------------------------------------------- */

/* Largest m accepted by lp_chol_solve_noalloc. */
#define LP_NOALLOC_MAX_M 32768

/* lp_chol_solve for callers that cannot allocate device memory or supply a
 * workspace (code under stream capture, serving loops that forbid
 * allocation): dy = L^-T L^-1 r with the same kernels and the same result as
 * lp_chol_solve, its scratch (about 260 KiB: the triangular solves' tickets
 * and flags and z = L^-1 r) taken from a fixed device array that the library
 * holds on every GPU it runs on until the process ends.  L (device,
 * row-major lower, ldm >= m), r and dy (device m-vectors, not aliased).
 * Errors: LP_ERR_INVALID_ARG (NULL, aliasing, ldm < m), LP_ERR_SHAPE
 * (m < 1), LP_ERR_WORKSPACE (m > LP_NOALLOC_MAX_M), LP_ERR_DEVICE.  Calls no
 * allocator; stream-ordered, does not synchronise.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (several
 * streams or host threads) race and must be serialised by the caller. */
lp_status lp_chol_solve_noalloc(int64_t m, const double* L, int64_t ldm, const double* r,
                                double* dy, lp_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* PDAS_H */
