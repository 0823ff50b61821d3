/*
 * pdas_oracle.c -- plain CPU oracle for Primal-Dual Affine Scaling (PDAS).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU library never
 * links, includes or calls it, and it shares no code, header or constant with
 * the GPU path.
 *
 * Source: N. Divakar, "Primal Dual Affine Scaling on GPUs", arXiv 1502.03543.
 *   - primal/dual pair: Section 1, equations (primal) and (dual);
 *   - KKT conditions and the Newton system: Section 3, equation (bigsystem);
 *   - the outer loop: Section 3, Algorithm "Primal-Dual Affine Scaling";
 *   - the reduction to normal equations (ADA^T) dy = ... with D = S^-1 X:
 *     Section 5, equation (bigsystem2) and the component formulas under it;
 *   - Cholesky of ADA^T: Section 5.1 (named there as the usual method);
 *   - the predictor-corrector variant at the end of this file: Mehrotra's
 *     method, which Section 4 (previous work) cites, on the same system.
 *
 * Readings taken where the paper is silent or garbled (each listed in the
 * design notes of the repository):
 *   R1  residual form.  The right-hand side of the Newton system is
 *       [r_p; r_d; -Xs] with r_p = b - Ax and r_d = c - A^T y - s; eliminating
 *       dx and ds gives (A D A^T) dy = b + A (d o r_d), ds = r_d - A^T dy,
 *       dx = -x - d o ds.  On a feasible iterate (r_p = r_d = 0) this is the
 *       paper's (ADA^T) dy = Ax, ds = -A^T dy, dx = D(-ds) - x.
 *   R2  psi == 1 is tested with exact floating-point equality, as written.
 *   R3  "optimum" after the psi == 1 step refers to the updated iterate.
 *   R4  the zero-direction test is kept literally (exact zeros).
 *   R5  the endless loop stops when the duality gap x^T s falls below a
 *       tolerance, tested before each direction; at most max_iter directions.
 *   R6  argmax tie-break: first index, x-block before s-block.
 *   R7  a non-positive or non-finite Cholesky pivot ends the run with a
 *       breakdown status and the last valid iterate (no silent fallback).
 *   R8  a non-finite or non-positive psi ends the run (it cannot happen in
 *       exact arithmetic: u_j + v_j = -1 forces psi >= 1/2).
 *
 * Arithmetic: REAL is double (liboracle_f64) or long double (liboracle_f80).
 * Every loop is the textbook definition, summing in index order; the build
 * disables floating-point contraction.  The only parallelism is OpenMP over
 * independent output rows, which leaves each element's summation order intact.
 *
 * Layouts: A is row-major m x n (A[i*n + j]); M and L are row-major m x m.
 */
#include <tgmath.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef REAL
#define REAL double
#endif

typedef REAL real;

/* Status codes of the oracle (its own numbering). */
enum {
  ORC_CONTINUE = 0,
  ORC_CONVERGED = 1,
  ORC_OPTIMAL_PSI1 = 2,
  ORC_OPTIMAL_ZERO_DIR = 3,
  ORC_MAX_ITER = 4,
  ORC_ERR_INVALID_ARG = -1,
  ORC_ERR_SHAPE = -2,
  ORC_ERR_NOT_INTERIOR = -3,
  ORC_ERR_BREAKDOWN = -4,
  ORC_ERR_NONPOS_PSI = -5,
  ORC_ERR_LOST_INTERIOR = -6
};

/* Intermediates of one iteration; every pointer may be NULL. */
typedef struct {
  double* r_d;  /* n: c - A^T y - s                                 */
  double* r_p;  /* m: b - A x                                       */
  double* d;    /* n: x / s                                         */
  double* M;    /* m*m: A diag(d) A^T, both triangles               */
  double* L;    /* m*m: Cholesky factor, lower, zeros above         */
  double* rhs;  /* m: b + A (d o r_d)                               */
  double* dx;   /* n */
  double* dy;   /* m */
  double* ds;   /* n */
  double gap;   /* x^T s of the input iterate                       */
  double psi;
  double t;         /* alpha_eff / psi                              */
  double alpha_eff;
  long long argmax; /* j in [0,n): x-block; n + j: s-block           */
  double min_pivot; /* smallest squared diagonal of L               */
  long long fail_col;  /* first failing pivot column, or -1         */
} orc_iter_out;

/* Per-iteration log of orc_solve. */
typedef struct {
  double gap;      /* before the step */
  double psi;
  double t;
  long long argmax;
  double rp_norm;  /* ||b - A x||_2 before the step */
  double rd_norm;  /* ||c - A^T y - s||_2 before the step */
  double min_pivot;
} orc_log;

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int orc_real_bytes(void) { return (int)sizeof(real); }

/* ------------------------------------------------------------------ */
/* Building blocks: each is the plain definition.                     */
/* ------------------------------------------------------------------ */

/* y = A^T v  (n outputs), Section 5 component formulas. */
static void at_times(long m, long n, const real* A, const real* v, real* out) {
  for (long j = 0; j < n; ++j) {
    real acc = 0;
    for (long i = 0; i < m; ++i) acc += A[i * n + j] * v[i];
    out[j] = acc;
  }
}

/* y = A v  (m outputs). */
static void a_times(long m, long n, const real* A, const real* v, real* out) {
  for (long i = 0; i < m; ++i) {
    real acc = 0;
    for (long j = 0; j < n; ++j) acc += A[i * n + j] * v[j];
    out[i] = acc;
  }
}

/* M = A diag(d) A^T, Section 5: the normal matrix of the reduced system.
 * M_ik = sum_j A_ij d_j A_kj.  Full symmetric matrix, lower computed and
 * mirrored. */
static void normal_matrix(long m, long n, const real* A, const real* d, real* M) {
#pragma omp parallel for schedule(dynamic, 4)
  for (long i = 0; i < m; ++i) {
    for (long k = 0; k <= i; ++k) {
      real acc = 0;
      for (long j = 0; j < n; ++j) acc += A[i * n + j] * d[j] * A[k * n + j];
      M[i * m + k] = acc;
    }
  }
  for (long i = 0; i < m; ++i)
    for (long k = i + 1; k < m; ++k) M[i * m + k] = M[k * m + i];
}

/* Cholesky M = L L^T (Section 5.1), column by column:
 *   L_jj = sqrt(M_jj - sum_{k<j} L_jk^2),
 *   L_ij = (M_ij - sum_{k<j} L_ik L_jk) / L_jj   for i > j.
 * Returns -1 on success, else the first column whose pivot is not a finite
 * positive number.  *min_pivot receives the smallest accepted pivot. */
static long cholesky(long m, const real* M, real* L, real* min_pivot) {
  for (long i = 0; i < m * m; ++i) L[i] = 0;
  real minp = INFINITY;
  for (long j = 0; j < m; ++j) {
    real p = M[j * m + j];
    for (long k = 0; k < j; ++k) p -= L[j * m + k] * L[j * m + k];
    if (!(p > 0) || !isfinite(p)) {
      *min_pivot = minp;
      return j;
    }
    if (p < minp) minp = p;
    real ljj = sqrt(p);
    L[j * m + j] = ljj;
#pragma omp parallel for schedule(static) if (m - j > 256)
    for (long i = j + 1; i < m; ++i) {
      real acc = M[i * m + j];
      for (long k = 0; k < j; ++k) acc -= L[i * m + k] * L[j * m + k];
      L[i * m + j] = acc / ljj;
    }
  }
  *min_pivot = minp;
  return -1;
}

/* Forward substitution L z = r, then back substitution L^T w = z. */
static void cholesky_solve(long m, const real* L, const real* r, real* w) {
  real* z = (real*)malloc(sizeof(real) * (size_t)m);
  for (long i = 0; i < m; ++i) {
    real acc = r[i];
    for (long k = 0; k < i; ++k) acc -= L[i * m + k] * z[k];
    z[i] = acc / L[i * m + i];
  }
  for (long i = m - 1; i >= 0; --i) {
    real acc = z[i];
    for (long k = i + 1; k < m; ++k) acc -= L[k * m + i] * w[k];
    w[i] = acc / L[i * m + i];
  }
  free(z);
}

static real dot(long n, const real* a, const real* b) {
  real acc = 0;
  for (long j = 0; j < n; ++j) acc += a[j] * b[j];
  return acc;
}

static real norm2(long n, const real* a) { return sqrt(dot(n, a, a)); }

static int all_finite(long n, const double* v) {
  for (long j = 0; j < n; ++j)
    if (!isfinite(v[j])) return 0;
  return 1;
}

/* ------------------------------------------------------------------ */
/* Working state                                                      */
/* ------------------------------------------------------------------ */

typedef struct {
  long m, n;
  real *A, *b, *c;        /* problem, converted to REAL */
  real *x, *y, *s;        /* current iterate            */
  real *rd, *rp, *d, *M, *L, *rhs, *dx, *dy, *ds, *g;
} state;

static void state_free(state* S) {
  real** p[] = {&S->A, &S->b, &S->c, &S->x, &S->y, &S->s, &S->rd, &S->rp, &S->d,
                &S->M, &S->L, &S->rhs, &S->dx, &S->dy, &S->ds, &S->g};
  for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); ++i) {
    free(*p[i]);
    *p[i] = NULL;
  }
}

static int state_alloc(state* S, long m, long n) {
  memset(S, 0, sizeof(*S));
  S->m = m;
  S->n = n;
  size_t mm = (size_t)m, nn = (size_t)n;
  S->A = malloc(sizeof(real) * mm * nn);
  S->b = malloc(sizeof(real) * mm);
  S->c = malloc(sizeof(real) * nn);
  S->x = malloc(sizeof(real) * nn);
  S->y = malloc(sizeof(real) * mm);
  S->s = malloc(sizeof(real) * nn);
  S->rd = malloc(sizeof(real) * nn);
  S->rp = malloc(sizeof(real) * mm);
  S->d = malloc(sizeof(real) * nn);
  S->M = malloc(sizeof(real) * mm * mm);
  S->L = malloc(sizeof(real) * mm * mm);
  S->rhs = malloc(sizeof(real) * mm);
  S->dx = malloc(sizeof(real) * nn);
  S->dy = malloc(sizeof(real) * mm);
  S->ds = malloc(sizeof(real) * nn);
  S->g = malloc(sizeof(real) * nn);
  if (!S->A || !S->b || !S->c || !S->x || !S->y || !S->s || !S->rd || !S->rp || !S->d ||
      !S->M || !S->L || !S->rhs || !S->dx || !S->dy || !S->ds || !S->g) {
    state_free(S);
    return 0;
  }
  return 1;
}

static void load(real* dst, const double* src, long k) {
  for (long i = 0; i < k; ++i) dst[i] = (real)src[i];
}
static void store(double* dst, const real* src, long k) {
  if (dst)
    for (long i = 0; i < k; ++i) dst[i] = (double)src[i];
}

/* Input validation, Section 1 (m < n, A full rank) and the interior start of
 * the Algorithm (x > 0, s > 0), 0 < alpha < 1. */
static int validate(long m, long n, const double* A, const double* b, const double* c,
                    const double* x, const double* y, const double* s, double alpha) {
  if (m < 1 || n < 1 || m >= n) return ORC_ERR_SHAPE;
  if (!A || !b || !c || !x || !y || !s) return ORC_ERR_INVALID_ARG;
  if (!(alpha > 0 && alpha < 1)) return ORC_ERR_INVALID_ARG;
  if (!all_finite(m * n, A) || !all_finite(m, b) || !all_finite(n, c) || !all_finite(n, x) ||
      !all_finite(m, y) || !all_finite(n, s))
    return ORC_ERR_INVALID_ARG;
  for (long j = 0; j < n; ++j)
    if (!(x[j] > 0) || !(s[j] > 0)) return ORC_ERR_NOT_INTERIOR;
  return ORC_CONTINUE;
}

/* One pass of the loop body of the Algorithm on state S (steps after the
 * gap test).  Fills psi/t/argmax/min_pivot/fail_col.  Updates x, y, s unless
 * an error occurs before the update. */
typedef struct {
  real psi, t, alpha_eff, min_pivot;
  long argmax, fail_col;
} step_info;

static int iterate_state(state* S, real alpha, step_info* info) {
  const long m = S->m, n = S->n;
  real* A = S->A;
  info->fail_col = -1;
  info->argmax = -1;
  info->psi = NAN;
  info->t = NAN;
  info->alpha_eff = alpha;
  info->min_pivot = NAN;

  /* Residuals (R1): r_d = c - A^T y - s and r_p = b - A x. */
  at_times(m, n, A, S->y, S->g);
  for (long j = 0; j < n; ++j) S->rd[j] = S->c[j] - S->g[j] - S->s[j];
  a_times(m, n, A, S->x, S->rp);
  for (long i = 0; i < m; ++i) S->rp[i] = S->b[i] - S->rp[i];

  /* D = S^-1 X (Section 5). */
  for (long j = 0; j < n; ++j) S->d[j] = S->x[j] / S->s[j];

  /* Normal matrix and right-hand side (R1). */
  normal_matrix(m, n, A, S->d, S->M);
  {
    real* t = S->g; /* reuse as d o r_d */
    for (long j = 0; j < n; ++j) t[j] = S->d[j] * S->rd[j];
    a_times(m, n, A, t, S->rhs);
    for (long i = 0; i < m; ++i) S->rhs[i] = S->b[i] + S->rhs[i];
  }

  /* Cholesky and the two triangular solves (Section 5.1). */
  long fail = cholesky(m, S->M, S->L, &info->min_pivot);
  if (fail >= 0) {
    info->fail_col = fail;
    return ORC_ERR_BREAKDOWN;
  }
  cholesky_solve(m, S->L, S->rhs, S->dy);

  /* ds = r_d - A^T dy; dx = -x - d o ds (Section 5 component formulas). */
  at_times(m, n, A, S->dy, S->g);
  for (long j = 0; j < n; ++j) S->ds[j] = S->rd[j] - S->g[j];
  for (long j = 0; j < n; ++j) S->dx[j] = -S->x[j] - S->d[j] * S->ds[j];

  /* Zero-direction stop (R4). */
  {
    int zero = 1;
    for (long j = 0; j < n && zero; ++j)
      if (S->dx[j] != 0 || S->ds[j] != 0) zero = 0;
    for (long i = 0; i < m && zero; ++i)
      if (S->dy[i] != 0) zero = 0;
    if (zero) return ORC_OPTIMAL_ZERO_DIR;
  }

  /* Ratio test: psi = max{ max_j(-dx_j/x_j), max_j(-ds_j/s_j) } (R6 ties). */
  real psi = -INFINITY;
  long arg = -1;
  for (long j = 0; j < n; ++j) {
    real u = -S->dx[j] / S->x[j];
    if (u > psi || arg < 0) { psi = u; arg = j; }
  }
  for (long j = 0; j < n; ++j) {
    real v = -S->ds[j] / S->s[j];
    if (v > psi) { psi = v; arg = n + j; }
  }
  info->psi = psi;
  info->argmax = arg;
  if (!isfinite(psi) || !(psi > 0)) return ORC_ERR_NONPOS_PSI;

  /* Step length (R2) and update. */
  real aeff = (psi == 1) ? (real)1 : alpha;
  real t = aeff / psi;
  info->alpha_eff = aeff;
  info->t = t;
  for (long j = 0; j < n; ++j) S->x[j] = S->x[j] + t * S->dx[j];
  for (long i = 0; i < m; ++i) S->y[i] = S->y[i] + t * S->dy[i];
  for (long j = 0; j < n; ++j) S->s[j] = S->s[j] + t * S->ds[j];

  if (psi == 1) return ORC_OPTIMAL_PSI1;
  for (long j = 0; j < n; ++j)
    if (!(S->x[j] > 0) || !(S->s[j] > 0)) return ORC_ERR_LOST_INTERIOR;
  return ORC_CONTINUE;
}

static void state_load(state* S, const double* A, const double* b, const double* c,
                       const double* x, const double* y, const double* s) {
  load(S->A, A, S->m * S->n);
  load(S->b, b, S->m);
  load(S->c, c, S->n);
  load(S->x, x, S->n);
  load(S->y, y, S->m);
  load(S->s, s, S->n);
}

/* ------------------------------------------------------------------ */
/* Exported entry points                                              */
/* ------------------------------------------------------------------ */

/* One iteration from (x, y, s), which are updated in place.  Returns an
 * ORC_* status (ORC_CONTINUE when the loop would go on). */
int orc_iterate(long m, long n, const double* A, const double* b, const double* c,
                double* x, double* y, double* s, double alpha, orc_iter_out* out) {
  int st = validate(m, n, A, b, c, x, y, s, alpha);
  if (st != ORC_CONTINUE) return st;
  state S;
  if (!state_alloc(&S, m, n)) return ORC_ERR_INVALID_ARG;
  state_load(&S, A, b, c, x, y, s);
  real gap = dot(n, S.x, S.s);
  step_info info;
  st = iterate_state(&S, (real)alpha, &info);
  if (out) {
    out->gap = (double)gap;
    out->psi = (double)info.psi;
    out->t = (double)info.t;
    out->alpha_eff = (double)info.alpha_eff;
    out->argmax = info.argmax;
    out->min_pivot = (double)info.min_pivot;
    out->fail_col = info.fail_col;
    store(out->r_d, S.rd, n);
    store(out->r_p, S.rp, m);
    store(out->d, S.d, n);
    store(out->M, S.M, m * m);
    if (st != ORC_ERR_BREAKDOWN) {
      store(out->L, S.L, m * m);
      store(out->rhs, S.rhs, m);
      store(out->dx, S.dx, n);
      store(out->dy, S.dy, m);
      store(out->ds, S.ds, n);
    }
  }
  if (st == ORC_CONTINUE || st == ORC_OPTIMAL_PSI1 || st == ORC_ERR_LOST_INTERIOR) {
    store(x, S.x, n);
    store(y, S.y, m);
    store(s, S.s, n);
  }
  state_free(&S);
  return st;
}

/* The Algorithm's loop (R5): before each direction, stop if x^T s < gap_tol,
 * or if max_iter directions have been taken.  (x, y, s) in/out receive the
 * last valid iterate.  log (max_iter entries) and tape ((max_iter+1) rows of
 * [x (n) | y (m) | s (n)]) may be NULL; tape row k is the iterate before
 * direction k.  *iters receives the number of steps taken. */
int orc_solve(long m, long n, const double* A, const double* b, const double* c,
              double* x, double* y, double* s, double alpha, double gap_tol, int max_iter,
              int* iters, orc_log* log, double* tape) {
  int st = validate(m, n, A, b, c, x, y, s, alpha);
  if (iters) *iters = 0;
  if (st != ORC_CONTINUE) return st;
  if (max_iter < 0) return ORC_ERR_INVALID_ARG;
  state S;
  if (!state_alloc(&S, m, n)) return ORC_ERR_INVALID_ARG;
  state_load(&S, A, b, c, x, y, s);
  const long row = 2 * n + m;
  int k = 0;
  for (;;) {
    if (tape) {
      store(tape + (size_t)k * row, S.x, n);
      store(tape + (size_t)k * row + n, S.y, m);
      store(tape + (size_t)k * row + n + m, S.s, n);
    }
    real gap = dot(n, S.x, S.s);
    if (gap < (real)gap_tol) { st = ORC_CONVERGED; break; }
    if (k >= max_iter) { st = ORC_MAX_ITER; break; }
    /* keep a copy of the iterate so an error leaves the last valid one */
    real* keep = malloc(sizeof(real) * (size_t)row);
    memcpy(keep, S.x, sizeof(real) * n);
    memcpy(keep + n, S.y, sizeof(real) * m);
    memcpy(keep + n + m, S.s, sizeof(real) * n);
    step_info info;
    st = iterate_state(&S, (real)alpha, &info);
    if (log) {
      log[k].gap = (double)gap;
      log[k].psi = (double)info.psi;
      log[k].t = (double)info.t;
      log[k].argmax = info.argmax;
      log[k].rp_norm = (double)norm2(m, S.rp);
      log[k].rd_norm = (double)norm2(n, S.rd);
      log[k].min_pivot = (double)info.min_pivot;
    }
    if (st == ORC_ERR_LOST_INTERIOR) {
      memcpy(S.x, keep, sizeof(real) * n);
      memcpy(S.y, keep + n, sizeof(real) * m);
      memcpy(S.s, keep + n + m, sizeof(real) * n);
    }
    free(keep);
    if (st == ORC_CONTINUE) { ++k; continue; }
    if (st == ORC_OPTIMAL_PSI1) ++k;
    break;
  }
  if (iters) *iters = k;
  store(x, S.x, n);
  store(y, S.y, m);
  store(s, S.s, n);
  state_free(&S);
  return st;
}

/* Fixed-K forward run from a perturbed start, in REAL precision, for
 * finite differences: the inputs are (A + h dA, b + h db, c + h dc,
 * x0 + h dx0, y0 + h dy0, s0 + h ds0) formed in REAL; any direction may be
 * NULL (zero).  Runs exactly K directions unless the loop stops first, and
 * returns w^T x_K in *loss.  Returns the status of the last step
 * (ORC_CONTINUE when all K steps ran). */
int orc_forward_k(long m, long n, const double* A, const double* b, const double* c,
                  const double* x0, const double* y0, const double* s0, double alpha, int K,
                  const double* dA, const double* db, const double* dc, const double* dx0,
                  const double* dy0, const double* ds0, double h, const double* w,
                  double* loss, double* xK, double* yK, double* sK) {
  int st = validate(m, n, A, b, c, x0, y0, s0, alpha);
  if (st != ORC_CONTINUE) return st;
  state S;
  if (!state_alloc(&S, m, n)) return ORC_ERR_INVALID_ARG;
  state_load(&S, A, b, c, x0, y0, s0);
  real hh = (real)h;
  if (dA) for (long i = 0; i < m * n; ++i) S.A[i] += hh * (real)dA[i];
  if (db) for (long i = 0; i < m; ++i) S.b[i] += hh * (real)db[i];
  if (dc) for (long j = 0; j < n; ++j) S.c[j] += hh * (real)dc[j];
  if (dx0) for (long j = 0; j < n; ++j) S.x[j] += hh * (real)dx0[j];
  if (dy0) for (long i = 0; i < m; ++i) S.y[i] += hh * (real)dy0[i];
  if (ds0) for (long j = 0; j < n; ++j) S.s[j] += hh * (real)ds0[j];
  st = ORC_CONTINUE;
  for (int k = 0; k < K && st == ORC_CONTINUE; ++k) {
    step_info info;
    st = iterate_state(&S, (real)alpha, &info);
  }
  if (loss && w) {
    real acc = 0;
    for (long j = 0; j < n; ++j) acc += (real)w[j] * S.x[j];
    *loss = (double)acc;
  }
  store(xK, S.x, n);
  store(yK, S.y, m);
  store(sK, S.s, n);
  state_free(&S);
  return st;
}

/* Reverse mode through K recorded steps.  tape holds K+1 rows of
 * [x | y | s] as written by orc_solve (row k = iterate before step k); each
 * step is recomputed from its row.  The psi == 1 branch is treated as a
 * constant step length.  Seeds: xbar_K (n), ybar_K (m, may be NULL),
 * sbar_K (n, may be NULL).  Outputs (each may be NULL): Abar (m*n),
 * bbar (m), cbar (n), x0bar (n), y0bar (m), s0bar (n).
 *
 * For each step, with the step's own values (r_d, d, M = LL^T, dx, dy, ds,
 * psi, t, argmax j*), the chain rule through
 *   x' = x + t dx, y' = y + t dy, s' = s + t ds,  t = alpha/psi,
 *   psi = -dx[J] / x[J] (or -ds[J] / s[J]) at the argmax J,  dx = -x - d o ds,
 *   ds = r_d - A^T dy,  M dy = rhs,  M = A D A^T,  rhs = b + A (d o r_d),
 *   d = x / s,  r_d = c - A^T y - s
 * is applied in reverse order. */
int orc_backward(long m, long n, const double* A, const double* b, const double* c,
                 double alpha, int K, const double* tape, const double* xbar_K,
                 const double* ybar_K, const double* sbar_K, double* Abar, double* bbar,
                 double* cbar, double* x0bar, double* y0bar, double* s0bar) {
  if (m < 1 || n <= m || K < 0 || !tape || !xbar_K) return ORC_ERR_INVALID_ARG;
  state S;
  if (!state_alloc(&S, m, n)) return ORC_ERR_INVALID_ARG;
  size_t mm = (size_t)m, nn = (size_t)n;
  real* xb = calloc(nn, sizeof(real));
  real* yb = calloc(mm, sizeof(real));
  real* sb = calloc(nn, sizeof(real));
  real* Ab = calloc(mm * nn, sizeof(real));
  real* bb = calloc(mm, sizeof(real));
  real* cb = calloc(nn, sizeof(real));
  real* dxb = malloc(sizeof(real) * nn);
  real* dyb = malloc(sizeof(real) * mm);
  real* dsb = malloc(sizeof(real) * nn);
  real* db_ = malloc(sizeof(real) * nn);
  real* rdb = malloc(sizeof(real) * nn);
  real* lam = malloc(sizeof(real) * mm);
  real* h = malloc(sizeof(real) * nn);
  real* tmpm = malloc(sizeof(real) * mm);
  load(xb, xbar_K, n);
  if (ybar_K) load(yb, ybar_K, m);
  if (sbar_K) load(sb, sbar_K, n);
  load(S.A, A, m * n);
  load(S.b, b, m);
  load(S.c, c, n);
  const long row = 2 * n + m;
  int st = ORC_CONTINUE;
  for (int k = K - 1; k >= 0; --k) {
    const double* it = tape + (size_t)k * row;
    load(S.x, it, n);
    load(S.y, it + n, m);
    load(S.s, it + n + m, n);
    real* x = malloc(sizeof(real) * nn);
    real* y = malloc(sizeof(real) * mm);
    real* s = malloc(sizeof(real) * nn);
    memcpy(x, S.x, sizeof(real) * nn);
    memcpy(y, S.y, sizeof(real) * mm);
    memcpy(s, S.s, sizeof(real) * nn);
    step_info info;
    int fst = iterate_state(&S, (real)alpha, &info); /* recompute the step */
    if (fst != ORC_CONTINUE && fst != ORC_OPTIMAL_PSI1) {
      free(x); free(y); free(s);
      st = fst;
      break;
    }
    const real t = info.t, psi = info.psi, aeff = info.alpha_eff;
    const long js = info.argmax;
    /* g = A^T dy (recomputed; S.g held d o r_d scratch then A^T dy) */
    real* g = S.g;
    at_times(m, n, S.A, S.dy, g);

    /* x' = x + t dx etc. */
    real tb = dot(n, xb, S.dx) + dot(m, yb, S.dy) + dot(n, sb, S.ds);
    for (long j = 0; j < n; ++j) dxb[j] = t * xb[j];
    for (long i = 0; i < m; ++i) dyb[i] = t * yb[i];
    for (long j = 0; j < n; ++j) dsb[j] = t * sb[j];
    /* t = alpha_eff / psi */
    real psib = -aeff * tb / (psi * psi);
    /* psi = -dx_j/x_j  or  -ds_j/s_j */
    if (js < n) {
      dxb[js] += -psib / x[js];
      xb[js] += psib * S.dx[js] / (x[js] * x[js]);
    } else {
      long j = js - n;
      dsb[j] += -psib / s[j];
      sb[j] += psib * S.ds[j] / (s[j] * s[j]);
    }
    /* dx = -x - d o ds */
    for (long j = 0; j < n; ++j) {
      xb[j] -= dxb[j];
      db_[j] = -dxb[j] * S.ds[j];
      dsb[j] -= S.d[j] * dxb[j];
    }
    /* ds = r_d - g,  g = A^T dy */
    for (long j = 0; j < n; ++j) rdb[j] = dsb[j];
    a_times(m, n, S.A, dsb, tmpm);
    for (long i = 0; i < m; ++i) dyb[i] -= tmpm[i];
    /* dy = M^-1 rhs: lambda = M^-1 dybar (M symmetric) */
    cholesky_solve(m, S.L, dyb, lam);
    at_times(m, n, S.A, lam, h);
    /* M = A D A^T: Mbar = -lambda dy^T */
    for (long j = 0; j < n; ++j) db_[j] -= h[j] * g[j];
    /* rhs = b + A (d o r_d) */
    for (long i = 0; i < m; ++i) bb[i] += lam[i];
    for (long j = 0; j < n; ++j) {
      db_[j] += S.rd[j] * h[j];
      rdb[j] += S.d[j] * h[j];
    }
    /* Abar contributions of this step:
     *   -dy dsbar^T                (from g = A^T dy)
     *   -(lambda g^T + dy h^T) D   (from M)
     *   +lambda (d o r_d)^T        (from rhs)
     *   -y rdbar^T                 (from r_d), rdbar complete below   */
    /* d = x / s */
    for (long j = 0; j < n; ++j) {
      xb[j] += db_[j] / s[j];
      sb[j] -= db_[j] * x[j] / (s[j] * s[j]);
    }
    /* r_d = c - A^T y - s */
    for (long j = 0; j < n; ++j) {
      cb[j] += rdb[j];
      sb[j] -= rdb[j];
    }
    a_times(m, n, S.A, rdb, tmpm);
    for (long i = 0; i < m; ++i) yb[i] -= tmpm[i];
    for (long i = 0; i < m; ++i) {
      for (long j = 0; j < n; ++j) {
        real v = -S.dy[i] * dsb[j] - (lam[i] * g[j] + S.dy[i] * h[j]) * S.d[j] +
                 lam[i] * S.d[j] * S.rd[j] - y[i] * rdb[j];
        Ab[(size_t)i * nn + j] += v;
      }
    }
    free(x); free(y); free(s);
  }
  if (st == ORC_CONTINUE) {
    store(Abar, Ab, m * n);
    store(bbar, bb, m);
    store(cbar, cb, n);
    store(x0bar, xb, n);
    store(y0bar, yb, m);
    store(s0bar, sb, n);
  }
  free(xb); free(yb); free(sb); free(Ab); free(bb); free(cb);
  free(dxb); free(dyb); free(dsb); free(db_); free(rdb); free(lam); free(h); free(tmpm);
  state_free(&S);
  return st;
}

/* Forward mode (tangent) through K steps from the start point: given input
 * tangents (each may be NULL = zero), returns the tangents of x_K, y_K, s_K.
 * Derived independently of orc_backward by differentiating each formula of
 * the step in forward order; used for the dot-product test
 * <VJP(w), v> = <w, JVP(v)>. */
int orc_jvp(long m, long n, const double* A, const double* b, const double* c,
            const double* x0, const double* y0, const double* s0, double alpha, int K,
            const double* tA, const double* tb, const double* tc, const double* tx0,
            const double* ty0, const double* ts0, double* txK, double* tyK, double* tsK) {
  int st = validate(m, n, A, b, c, x0, y0, s0, alpha);
  if (st != ORC_CONTINUE) return st;
  state S;
  if (!state_alloc(&S, m, n)) return ORC_ERR_INVALID_ARG;
  state_load(&S, A, b, c, x0, y0, s0);
  size_t mm = (size_t)m, nn = (size_t)n;
  real* TA = calloc(mm * nn, sizeof(real));
  real* Tb = calloc(mm, sizeof(real));
  real* Tc = calloc(nn, sizeof(real));
  real* Tx = calloc(nn, sizeof(real));
  real* Ty = calloc(mm, sizeof(real));
  real* Ts = calloc(nn, sizeof(real));
  real* Trd = malloc(sizeof(real) * nn);
  real* Td = malloc(sizeof(real) * nn);
  real* Trhs = malloc(sizeof(real) * mm);
  real* Tdy = malloc(sizeof(real) * mm);
  real* Tg = malloc(sizeof(real) * nn);
  real* Tds = malloc(sizeof(real) * nn);
  real* Tdx = malloc(sizeof(real) * nn);
  real* vn = malloc(sizeof(real) * nn);
  real* vn2 = malloc(sizeof(real) * nn);
  real* vm = malloc(sizeof(real) * mm);
  real* x = malloc(sizeof(real) * nn);
  real* s = malloc(sizeof(real) * nn);
  if (tA) load(TA, tA, m * n);
  if (tb) load(Tb, tb, m);
  if (tc) load(Tc, tc, n);
  if (tx0) load(Tx, tx0, n);
  if (ty0) load(Ty, ty0, m);
  if (ts0) load(Ts, ts0, n);
  st = ORC_CONTINUE;
  for (int k = 0; k < K && st == ORC_CONTINUE; ++k) {
    memcpy(x, S.x, sizeof(real) * nn);
    memcpy(s, S.s, sizeof(real) * nn);
    /* y before the step is needed: keep it in vm-sized copy */
    real* y = malloc(sizeof(real) * mm);
    memcpy(y, S.y, sizeof(real) * mm);
    step_info info;
    st = iterate_state(&S, (real)alpha, &info);
    if (st != ORC_CONTINUE && st != ORC_OPTIMAL_PSI1) { free(y); break; }
    real* g = S.g;
    at_times(m, n, S.A, S.dy, g);
    /* r_d = c - A^T y - s */
    at_times(m, n, TA, y, vn);
    at_times(m, n, S.A, Ty, vn2);
    for (long j = 0; j < n; ++j) Trd[j] = Tc[j] - vn[j] - vn2[j] - Ts[j];
    /* d = x / s */
    for (long j = 0; j < n; ++j) Td[j] = Tx[j] / s[j] - x[j] * Ts[j] / (s[j] * s[j]);
    /* rhs = b + A (d o r_d) */
    for (long j = 0; j < n; ++j) vn[j] = S.d[j] * S.rd[j];
    a_times(m, n, TA, vn, Trhs);
    for (long j = 0; j < n; ++j) vn[j] = Td[j] * S.rd[j] + S.d[j] * Trd[j];
    a_times(m, n, S.A, vn, vm);
    for (long i = 0; i < m; ++i) Trhs[i] = Tb[i] + Trhs[i] + vm[i];
    /* M dy = rhs  =>  M Tdy = Trhs - TM dy,
     * TM dy = TA (d o g) + A (Td o g) + A (d o (TA^T dy)) */
    for (long j = 0; j < n; ++j) vn[j] = S.d[j] * g[j];
    a_times(m, n, TA, vn, vm);
    for (long i = 0; i < m; ++i) Trhs[i] -= vm[i];
    at_times(m, n, TA, S.dy, vn2); /* TA^T dy */
    for (long j = 0; j < n; ++j) vn[j] = Td[j] * g[j] + S.d[j] * vn2[j];
    a_times(m, n, S.A, vn, vm);
    for (long i = 0; i < m; ++i) Trhs[i] -= vm[i];
    cholesky_solve(m, S.L, Trhs, Tdy);
    /* g = A^T dy,  ds = r_d - g,  dx = -x - d o ds */
    at_times(m, n, S.A, Tdy, Tg);
    for (long j = 0; j < n; ++j) Tg[j] += vn2[j];
    for (long j = 0; j < n; ++j) Tds[j] = Trd[j] - Tg[j];
    for (long j = 0; j < n; ++j) Tdx[j] = -Tx[j] - Td[j] * S.ds[j] - S.d[j] * Tds[j];
    /* psi at the recorded argmax, t = alpha_eff / psi */
    real Tpsi;
    long js = info.argmax;
    if (js < n)
      Tpsi = -Tdx[js] / x[js] + S.dx[js] * Tx[js] / (x[js] * x[js]);
    else {
      long j = js - n;
      Tpsi = -Tds[j] / s[j] + S.ds[j] * Ts[j] / (s[j] * s[j]);
    }
    real Tt = -info.alpha_eff * Tpsi / (info.psi * info.psi);
    for (long j = 0; j < n; ++j) Tx[j] += Tt * S.dx[j] + info.t * Tdx[j];
    for (long i = 0; i < m; ++i) Ty[i] += Tt * S.dy[i] + info.t * Tdy[i];
    for (long j = 0; j < n; ++j) Ts[j] += Tt * S.ds[j] + info.t * Tds[j];
    free(y);
    if (st == ORC_OPTIMAL_PSI1) break;
  }
  if (st == ORC_CONTINUE || st == ORC_OPTIMAL_PSI1) {
    store(txK, Tx, n);
    store(tyK, Ty, m);
    store(tsK, Ts, n);
  }
  free(TA); free(Tb); free(Tc); free(Tx); free(Ty); free(Ts); free(Trd); free(Td);
  free(Trhs); free(Tdy); free(Tg); free(Tds); free(Tdx); free(vn); free(vn2); free(vm);
  free(x); free(s);
  state_free(&S);
  return st;
}

/* Building blocks exported for unit pins. */
void orc_normal_matrix(long m, long n, const double* A, const double* d, double* M) {
  real* Ar = malloc(sizeof(real) * (size_t)m * n);
  real* dr = malloc(sizeof(real) * (size_t)n);
  real* Mr = malloc(sizeof(real) * (size_t)m * m);
  load(Ar, A, m * n);
  load(dr, d, n);
  normal_matrix(m, n, Ar, dr, Mr);
  store(M, Mr, m * m);
  free(Ar); free(dr); free(Mr);
}

long orc_cholesky(long m, const double* M, double* L, double* min_pivot) {
  real* Mr = malloc(sizeof(real) * (size_t)m * m);
  real* Lr = malloc(sizeof(real) * (size_t)m * m);
  real mp;
  load(Mr, M, m * m);
  long f = cholesky(m, Mr, Lr, &mp);
  store(L, Lr, m * m);
  if (min_pivot) *min_pivot = (double)mp;
  free(Mr); free(Lr);
  return f;
}

void orc_cholesky_solve(long m, const double* L, const double* r, double* w) {
  real* Lr = malloc(sizeof(real) * (size_t)m * m);
  real* rr = malloc(sizeof(real) * (size_t)m);
  real* wr = malloc(sizeof(real) * (size_t)m);
  load(Lr, L, m * m);
  load(rr, r, m);
  cholesky_solve(m, Lr, rr, wr);
  store(w, wr, m);
  free(Lr); free(rr); free(wr);
}

/* ------------------------------------------------------------------ */
/* Predictor-corrector variant (Mehrotra)                             */
/* ------------------------------------------------------------------ */
/*
 * The paper's Section 4 (previous work) cites Mehrotra's primal-dual method
 * as the second-order, centred refinement of the affine-scaling direction.
 * It is a different method from the Section 3 algorithm; this is its
 * published definition (Mehrotra, SIAM J. Optim. 2(4), 1992; as stated in
 * S. J. Wright, Primal-Dual Interior-Point Methods, SIAM 1997, ch. 10),
 * written out on the same Newton system (bigsystem) and the same Section 5
 * reduction, one factorization per iteration:
 *
 *   predictor: the Section 3 (affine-scaling) direction, third right-hand
 *              side r_c = -X S e;
 *   step to the boundary, primal and dual apart:
 *              a_max_p = min over dx_j < 0 of -x_j/dx_j (inf if none),
 *              a_aff_p = min(1, a_max_p), and a_aff_d the same with s, ds;
 *   centring:  mu = x^T s / n,
 *              mu_aff = (x + a_aff_p dx_aff)^T (s + a_aff_d ds_aff) / n,
 *              sigma = (mu_aff / mu)^3;
 *   corrector: the same system with r_c = -X S e - dX_aff dS_aff e
 *              + sigma mu e;
 *   step:      a_p = min(1, eta a_max_p), a_d = min(1, eta a_max_d) for the
 *              corrector direction; x += a_p dx, y += a_d dy, s += a_d ds.
 *
 * With D = S^-1 X and the residuals r_p = b - A x, r_d = c - A^T y - s,
 * eliminating dx and ds from (A dx = r_p, A^T dy + ds = r_d,
 * S dx + X ds = r_c) gives
 *   (A D A^T) dy = b + A (d o r_d - x - r_c / s),
 *   ds = r_d - A^T dy,   dx = r_c / s - d o ds;
 * for r_c = -X S e this is the Section 5 residual-form system (R1).
 */

typedef struct {
  double* dx_aff;  /* n, predictor direction (nullable) */
  double* dy_aff;  /* m */
  double* ds_aff;  /* n */
  double* dx;      /* n, corrector direction (nullable) */
  double* dy;      /* m */
  double* ds;      /* n */
  double* rhs_aff; /* m, right-hand sides of the two reduced solves */
  double* rhs;     /* m */
  double gap, mu, mu_aff, sigma;
  double alpha_aff_p, alpha_aff_d, alpha_p, alpha_d;
  double min_pivot;
  long long fail_col;
} orc_pc_out;

typedef struct {
  double gap;      /* before the step */
  double sigma;
  double alpha_p;
  double alpha_d;
  double min_pivot;
} orc_pc_log;

/* Largest step in [0, inf) keeping v + a dv >= 0: min over dv_j < 0 of
 * -v_j/dv_j, +inf when no component decreases. */
static real step_to_boundary(long n, const real* v, const real* dv) {
  real a = INFINITY;
  for (long j = 0; j < n; ++j)
    if (dv[j] < 0) {
      real r = -v[j] / dv[j];
      if (r < a) a = r;
    }
  return a;
}

/* Reduced solve for third right-hand side rc (n): dy, ds, dx into S (uses
 * the factor S->L and the dual residual S->rd already formed); rhs_out
 * receives the reduced right-hand side. */
static void pc_direction(state* S, const real* rc, real* rhs_out, real* dx, real* dy,
                         real* ds) {
  const long m = S->m, n = S->n;
  real* t = S->g;
  for (long j = 0; j < n; ++j) t[j] = S->d[j] * S->rd[j] - S->x[j] - rc[j] / S->s[j];
  a_times(m, n, S->A, t, rhs_out);
  for (long i = 0; i < m; ++i) rhs_out[i] = S->b[i] + rhs_out[i];
  cholesky_solve(m, S->L, rhs_out, dy);
  at_times(m, n, S->A, dy, S->g);
  for (long j = 0; j < n; ++j) ds[j] = S->rd[j] - S->g[j];
  for (long j = 0; j < n; ++j) dx[j] = rc[j] / S->s[j] - S->d[j] * ds[j];
}

typedef struct {
  real gap, mu, mu_aff, sigma, a_aff_p, a_aff_d, a_p, a_d, min_pivot;
  long fail_col;
} pc_info;

/* One predictor-corrector iteration on S; aux holds 3n + 2m + n reals for
 * the predictor direction, the corrector right-hand side and r_c. */
static int pc_iterate_state(state* S, real eta, real* aux, real* rhs_aff, pc_info* info) {
  const long m = S->m, n = S->n;
  real* dxa = aux;
  real* dya = aux + n;
  real* dsa = aux + n + m;
  real* rc = aux + 2 * n + m;
  info->fail_col = -1;
  info->sigma = NAN;
  info->a_p = info->a_d = NAN;
  info->min_pivot = NAN;
  info->gap = dot(n, S->x, S->s);
  info->mu = info->gap / (real)n;

  /* residual r_d = c - A^T y - s and D = S^-1 X (Section 5) */
  at_times(m, n, S->A, S->y, S->g);
  for (long j = 0; j < n; ++j) {
    const real aty = S->g[j];
    S->rd[j] = S->c[j] - aty - S->s[j];
  }
  for (long j = 0; j < n; ++j) {
    const real xj = S->x[j], sj = S->s[j];
    S->d[j] = xj / sj;
  }

  /* one normal matrix and one factor serve both solves */
  normal_matrix(m, n, S->A, S->d, S->M);
  long fail = cholesky(m, S->M, S->L, &info->min_pivot);
  if (fail >= 0) {
    info->fail_col = fail;
    return ORC_ERR_BREAKDOWN;
  }

  /* predictor: r_c = -X S e */
  for (long j = 0; j < n; ++j) rc[j] = -S->x[j] * S->s[j];
  pc_direction(S, rc, rhs_aff, dxa, dya, dsa);
  real ap = step_to_boundary(n, S->x, dxa), ad = step_to_boundary(n, S->s, dsa);
  info->a_aff_p = ap < 1 ? ap : (real)1;
  info->a_aff_d = ad < 1 ? ad : (real)1;
  real acc = 0;
  for (long j = 0; j < n; ++j)
    acc += (S->x[j] + info->a_aff_p * dxa[j]) * (S->s[j] + info->a_aff_d * dsa[j]);
  info->mu_aff = acc / (real)n;
  real q = info->mu_aff / info->mu;
  info->sigma = q * q * q;

  /* corrector: r_c = -X S e - dX_aff dS_aff e + sigma mu e */
  for (long j = 0; j < n; ++j)
    rc[j] = -S->x[j] * S->s[j] - dxa[j] * dsa[j] + info->sigma * info->mu;
  pc_direction(S, rc, S->rhs, S->dx, S->dy, S->ds);

  {
    int zero = 1;
    for (long j = 0; j < n && zero; ++j)
      if (S->dx[j] != 0 || S->ds[j] != 0) zero = 0;
    for (long i = 0; i < m && zero; ++i)
      if (S->dy[i] != 0) zero = 0;
    if (zero) return ORC_OPTIMAL_ZERO_DIR;
  }

  real mp = step_to_boundary(n, S->x, S->dx), md = step_to_boundary(n, S->s, S->ds);
  info->a_p = eta * mp < 1 ? eta * mp : (real)1;
  info->a_d = eta * md < 1 ? eta * md : (real)1;
  if (!(info->a_p > 0) || !(info->a_d > 0) || !isfinite(info->a_p) || !isfinite(info->a_d))
    return ORC_ERR_NONPOS_PSI;
  for (long j = 0; j < n; ++j) S->x[j] = S->x[j] + info->a_p * S->dx[j];
  for (long i = 0; i < m; ++i) S->y[i] = S->y[i] + info->a_d * S->dy[i];
  for (long j = 0; j < n; ++j) S->s[j] = S->s[j] + info->a_d * S->ds[j];
  for (long j = 0; j < n; ++j)
    if (!(S->x[j] > 0) || !(S->s[j] > 0)) return ORC_ERR_LOST_INTERIOR;
  return ORC_CONTINUE;
}

/* One predictor-corrector iteration from (x, y, s), updated in place
 * (eta in (0, 1): the fraction of the step to the boundary). */
int orc_pc_iterate(long m, long n, const double* A, const double* b, const double* c,
                   double* x, double* y, double* s, double eta, orc_pc_out* out) {
  int st = validate(m, n, A, b, c, x, y, s, eta);
  if (st != ORC_CONTINUE) return st;
  state S;
  if (!state_alloc(&S, m, n)) return ORC_ERR_INVALID_ARG;
  real* aux = malloc(sizeof(real) * (size_t)(3 * n + m));
  real* rhs_aff = malloc(sizeof(real) * (size_t)m);
  if (!aux || !rhs_aff) {
    free(aux);
    free(rhs_aff);
    state_free(&S);
    return ORC_ERR_INVALID_ARG;
  }
  state_load(&S, A, b, c, x, y, s);
  pc_info info;
  st = pc_iterate_state(&S, (real)eta, aux, rhs_aff, &info);
  if (out) {
    out->gap = (double)info.gap;
    out->mu = (double)info.mu;
    out->mu_aff = (double)info.mu_aff;
    out->sigma = (double)info.sigma;
    out->alpha_aff_p = (double)info.a_aff_p;
    out->alpha_aff_d = (double)info.a_aff_d;
    out->alpha_p = (double)info.a_p;
    out->alpha_d = (double)info.a_d;
    out->min_pivot = (double)info.min_pivot;
    out->fail_col = info.fail_col;
    if (st != ORC_ERR_BREAKDOWN) {
      store(out->dx_aff, aux, n);
      store(out->dy_aff, aux + n, m);
      store(out->ds_aff, aux + n + m, n);
      store(out->dx, S.dx, n);
      store(out->dy, S.dy, m);
      store(out->ds, S.ds, n);
      store(out->rhs_aff, rhs_aff, m);
      store(out->rhs, S.rhs, m);
    }
  }
  if (st == ORC_CONTINUE || st == ORC_ERR_LOST_INTERIOR) {
    store(x, S.x, n);
    store(y, S.y, m);
    store(s, S.s, n);
  }
  free(aux);
  free(rhs_aff);
  state_free(&S);
  return st;
}

/* The predictor-corrector loop: before each direction stop with
 * ORC_CONVERGED when x^T s < gap_tol, or ORC_MAX_ITER after max_iter
 * directions.  (x, y, s) in/out receive the last valid iterate; log
 * (max_iter entries) may be NULL. */
int orc_pc_solve(long m, long n, const double* A, const double* b, const double* c,
                 double* x, double* y, double* s, double eta, double gap_tol, int max_iter,
                 int* iters, orc_pc_log* log) {
  int st = validate(m, n, A, b, c, x, y, s, eta);
  if (iters) *iters = 0;
  if (st != ORC_CONTINUE) return st;
  if (max_iter < 0) return ORC_ERR_INVALID_ARG;
  state S;
  if (!state_alloc(&S, m, n)) return ORC_ERR_INVALID_ARG;
  const long row = 2 * n + m;
  real* aux = malloc(sizeof(real) * (size_t)(3 * n + m));
  real* rhs_aff = malloc(sizeof(real) * (size_t)m);
  real* keep = malloc(sizeof(real) * (size_t)row);
  if (!aux || !rhs_aff || !keep) {
    free(aux);
    free(rhs_aff);
    free(keep);
    state_free(&S);
    return ORC_ERR_INVALID_ARG;
  }
  state_load(&S, A, b, c, x, y, s);
  int k = 0;
  for (;;) {
    real gap = dot(n, S.x, S.s);
    if (gap < (real)gap_tol) { st = ORC_CONVERGED; break; }
    if (k >= max_iter) { st = ORC_MAX_ITER; break; }
    memcpy(keep, S.x, sizeof(real) * n);
    memcpy(keep + n, S.y, sizeof(real) * m);
    memcpy(keep + n + m, S.s, sizeof(real) * n);
    pc_info info;
    st = pc_iterate_state(&S, (real)eta, aux, rhs_aff, &info);
    if (log) {
      log[k].gap = (double)gap;
      log[k].sigma = (double)info.sigma;
      log[k].alpha_p = (double)info.a_p;
      log[k].alpha_d = (double)info.a_d;
      log[k].min_pivot = (double)info.min_pivot;
    }
    if (st == ORC_ERR_LOST_INTERIOR) {
      memcpy(S.x, keep, sizeof(real) * n);
      memcpy(S.y, keep + n, sizeof(real) * m);
      memcpy(S.s, keep + n + m, sizeof(real) * n);
    }
    if (st == ORC_CONTINUE) { ++k; continue; }
    break;
  }
  if (iters) *iters = k;
  store(x, S.x, n);
  store(y, S.y, m);
  store(s, S.s, n);
  free(aux);
  free(rhs_aff);
  free(keep);
  state_free(&S);
  return st;
}
