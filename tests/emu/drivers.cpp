// Host drivers for the emulated kernels (test infrastructure only).
//   emu chol <m> [g]                  lower Cholesky of a fixed SPD matrix with
//                                     one extra right-hand-side row; prints
//                                     the factor and forward-solve errors
//                                     against a long-double reference; g > 0
//                                     lowers the grouping threshold to g
//   emu syrk <m> <n> <tile> <splits>  normal matrix (tile 0: stream-K), against a
//                                     long-double reference
//   emu trsv <m>                      L z = r and L^T y = z with a fixed
//                                     lower-triangular L; prints both errors
//                                     against long-double substitution
//   emu sparse <m> <n> <pattern>      CSR check, CSC build, A w, A^T v and the
//                                     sparse normal matrix against long-double
//                                     references (pattern 0: a dense column,
//                                     an empty row and column, a row longer
//                                     than one metadata chunk; 1: uniform,
//                                     half full), then the check's verdict on
//                                     broken copies of the CSR
//   emu batch <in> <out> <max_iter> <tape> [tile] [mixed]
//                                     batched solve of the LPs in <in>; with a
//                                     tape, also the reverse sweep
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hip/hip_runtime.h"
#include "pdas_internal.h"

namespace pdas {
void launch_fill_i32(hipStream_t, int* p, int v, long count) {
  for (long i = 0; i < count; ++i) p[i] = v;
}
void launch_copy(hipStream_t, double* d, const double* s, long n) {
  std::memcpy(d, s, n * sizeof(double));
}
void launch_zero(hipStream_t, double* p, long n) {
  for (long i = 0; i < n; ++i) p[i] = 0.0;
}
}  // namespace pdas

extern "C" void lp_options_default(lp_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->alpha = 0.95;
  o->precision = LP_PREC_FP64;
  o->mixed_switch_gap = 1e-6;
  o->refine_tol = 0x1p-46;
  o->refine_max = 5;
}

// running maximum of errors in which a NaN (an entry never written, or
// garbage) counts as infinite; std::fmax would drop it
static double worse(double acc, double e) { return (e <= acc) ? acc : (std::isnan(e) ? INFINITY : e); }

static int run_chol(int m, int group_min_m) {
  // a lower grouping threshold takes small matrices through the grouped schedule
  if (group_min_m > 0) pdas::set_chol_group_min_m(group_min_m);
  const long ld = (m + 1 + 7) / 8 * 8;
  std::vector<double> A((size_t)(m + 1) * ld, NAN);  // upper part never read
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j)
      A[(size_t)i * ld + j] = (i == j) ? m : 0.5 / (1.0 + std::abs(i - j)) + 0.01 * ((i * 7 + j * 3) % 11);
  for (int j = 0; j < m; ++j) A[(size_t)m * ld + j] = std::cos(0.3 * j);
  std::vector<double> M = A, diag(pdas::potrf_diag_elems(m));
  pdas::DevInfo info{};
  info.chol_fail = INT_MAX;
  info.min_pivot = INFINITY;
  pdas::launch_potrf_f64(nullptr, m + 1, m, M.data(), ld, &info, diag.data());
  std::vector<long double> R((size_t)m * m, 0.0L);
  long double minp = INFINITY;
  for (int j = 0; j < m; ++j)
    for (int i = j; i < m; ++i) {
      long double s = A[(size_t)i * ld + j];
      for (int k = 0; k < j; ++k) s -= R[(size_t)i * m + k] * R[(size_t)j * m + k];
      if (i == j) minp = s < minp ? s : minp;
      R[(size_t)i * m + j] = (i == j) ? sqrtl(s) : s / R[(size_t)j * m + j];
    }
  double lerr = 0, lsc = 0, zerr = 0, zsc = 0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      lerr = worse(lerr, std::fabs((double)(M[(size_t)i * ld + j] - R[(size_t)i * m + j])));
      lsc = std::fmax(lsc, std::fabs((double)R[(size_t)i * m + j]));
    }
  std::vector<long double> z(m);
  for (int i = 0; i < m; ++i) {
    long double v = A[(size_t)m * ld + i];
    for (int k = 0; k < i; ++k) v -= R[(size_t)i * m + k] * z[k];
    z[i] = v / R[(size_t)i * m + i];
    zerr = worse(zerr, std::fabs((double)(z[i] - M[(size_t)m * ld + i])));
    zsc = std::fmax(zsc, std::fabs((double)z[i]));
  }
  const double perr = std::fabs((double)((info.min_pivot - minp) / minp));
  printf("{\"m\": %d, \"fail\": %d, \"factor_rel_err\": %.3e, \"solve_rel_err\": %.3e, "
         "\"min_pivot_rel_err\": %.3e}\n",
         m, info.chol_fail == INT_MAX ? -1 : info.chol_fail, lerr / lsc, zerr / zsc,
         std::isnan(perr) ? INFINITY : perr);
  return 0;
}

static int run_syrk(int m, int n, int tile, int splits) {
  std::vector<double> A((size_t)m * n), d(n);
  for (size_t i = 0; i < A.size(); ++i) A[i] = std::sin(0.7 * i + 0.3);
  for (int j = 0; j < n; ++j) d[j] = 0.5 + 0.25 * std::cos(1.3 * j);
  const long ldm = m + 3;
  std::vector<double> M((size_t)m * ldm, NAN);
  std::vector<double> part(pdas::syrk_part_elems(m, tile, splits) + 1, NAN);
  pdas::launch_syrk_f64(nullptr, m, n, A.data(), n, d.data(), M.data(), ldm, false, tile, splits,
                        (tile == 0 || splits > 1) ? part.data() : nullptr);
  double err = 0, sc = 0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      long double r = 0;
      for (int k = 0; k < n; ++k) r += (long double)A[(size_t)i * n + k] * d[k] * A[(size_t)j * n + k];
      err = worse(err, std::fabs((double)(M[(size_t)i * ldm + j] - r)));
      sc = std::fmax(sc, std::fabs((double)r));
    }
  printf("{\"m\": %d, \"n\": %d, \"tile\": %d, \"splits\": %d, \"rel_err\": %.3e}\n", m, n, tile,
         splits, err / sc);
  return 0;
}

static int run_trsv(int m) {
  const long ld = m + 5;
  const int nblk = (m + 63) / 64;
  std::vector<double> L((size_t)m * ld, NAN), r(m), z(m, NAN), y(m, NAN);
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < i; ++j) L[(size_t)i * ld + j] = 0.3 * std::sin(0.37 * i + 1.1 * j) / (1.0 + 0.05 * (i - j));
    L[(size_t)i * ld + i] = 1.5 + 0.5 * std::cos(0.9 * i);
    r[i] = std::cos(0.21 * i + 0.4);
  }
  std::vector<int> sync(4 + 2 * nblk, 0);
  pdas::DevInfo info{};
  pdas::launch_trsv_fwd(nullptr, m, L.data(), ld, r.data(), z.data(), sync.data(), &info);
  pdas::launch_trsv_bwd(nullptr, m, L.data(), ld, z.data(), y.data(), sync.data(), &info);
  std::vector<long double> zr(m), yr(m);
  for (int i = 0; i < m; ++i) {
    long double v = r[i];
    for (int k = 0; k < i; ++k) v -= (long double)L[(size_t)i * ld + k] * zr[k];
    zr[i] = v / L[(size_t)i * ld + i];
  }
  // the backward solve is checked on the device's z, so its error is its own
  for (int i = m - 1; i >= 0; --i) {
    long double v = z[i];
    for (int k = i + 1; k < m; ++k) v -= (long double)L[(size_t)k * ld + i] * yr[k];
    yr[i] = v / L[(size_t)i * ld + i];
  }
  double ze = 0, zs = 0, ye = 0, ys = 0;
  for (int i = 0; i < m; ++i) {
    ze = worse(ze, std::fabs((double)(z[i] - zr[i])));
    zs = std::fmax(zs, std::fabs((double)zr[i]));
    ye = worse(ye, std::fabs((double)(y[i] - yr[i])));
    ys = std::fmax(ys, std::fabs((double)yr[i]));
  }
  printf("{\"m\": %d, \"err_flag\": %d, \"fwd_rel_err\": %.3e, \"bwd_rel_err\": %.3e}\n", m,
         info.trsv_err, ze / zs, ye / ys);
  return 0;
}

static int run_batch(const char* in, const char* out, int max_iter, int tape, int tile,
                     int mixed) {
  FILE* f = fopen(in, "rb");
  if (!f) return 2;
  int count = 0;
  if (fread(&count, 4, 1, f) != 1) return 2;
  std::vector<int64_t> m(count), n(count), aoff(count), vom(count), von(count);
  std::vector<double> A, b, c, x0, y0, s0;
  for (int i = 0; i < count; ++i) {
    int64_t mn[2];
    if (fread(mn, 8, 2, f) != 2) return 2;
    m[i] = mn[0];
    n[i] = mn[1];
    aoff[i] = A.size();
    vom[i] = b.size();
    von[i] = c.size();
    auto rd = [&](std::vector<double>& v, long k) {
      const size_t o = v.size();
      v.resize(o + k);
      return fread(v.data() + o, 8, k, f) == (size_t)k;
    };
    if (!(rd(A, m[i] * n[i]) && rd(b, m[i]) && rd(c, n[i]) && rd(x0, n[i]) && rd(y0, m[i]) &&
          rd(s0, n[i])))
      return 2;
  }
  fclose(f);
  lp_options opt;
  lp_options_default(&opt);
  opt.tape_capacity = tape;
  opt.batch_tile = tile;
  if (mixed) opt.precision = LP_PREC_MIXED;
  size_t bytes = 0;
  int st = lp_batch_workspace_size(count, m.data(), n.data(), &opt, &bytes);
  if (st != LP_OK) return 3;
  void* ws = aligned_alloc(256, (bytes + 255) / 256 * 256);
  std::memset(ws, 0xff, bytes);  // NaN patterns, as an uninitialised pool might hold
  lp_batch* h = nullptr;
  st = lp_batch_setup(&h, count, m.data(), n.data(), A.data(), aoff.data(), b.data(), c.data(),
                      x0.data(), y0.data(), s0.data(), vom.data(), von.data(), &opt, ws, bytes,
                      nullptr);
  if (st != LP_OK) return 4;
  std::vector<int32_t> status(count), iters(count);
  int nconv = 0;
  st = lp_batch_solve(h, tape > 0 ? 0.0 : 1e-8, max_iter, status.data(), iters.data(), &nconv);
  if (st != LP_OK) return 5;
  std::vector<double> x(c.size()), y(b.size()), s(c.size());
  lp_batch_get_iterate(h, x.data(), y.data(), s.data());
  FILE* o = fopen(out, "wb");
  fwrite(status.data(), 4, count, o);
  fwrite(iters.data(), 4, count, o);
  fwrite(x.data(), 8, x.size(), o);
  fwrite(y.data(), 8, y.size(), o);
  fwrite(s.data(), 8, s.size(), o);
  if (tape > 0) {
    std::vector<double> xb(c.size()), Ab(A.size()), bb(b.size()), cb(c.size());
    for (size_t j = 0; j < xb.size(); ++j) xb[j] = std::sin(0.37 * j + 0.1);
    st = lp_batch_backward(h, xb.data(), nullptr, nullptr, Ab.data(), bb.data(), cb.data(),
                           nullptr, nullptr, nullptr);
    if (st != LP_OK) return 6;
    fwrite(Ab.data(), 8, Ab.size(), o);
    fwrite(bb.data(), 8, bb.size(), o);
    fwrite(cb.data(), 8, cb.size(), o);
    for (int k = 0; k < tape; ++k) {
      std::vector<double> tx(c.size()), ty(b.size()), ts(c.size());
      lp_batch_tape_row(h, k, tx.data(), ty.data(), ts.data());
      fwrite(tx.data(), 8, tx.size(), o);
      fwrite(ty.data(), 8, ty.size(), o);
      fwrite(ts.data(), 8, ts.size(), o);
    }
  }
  fclose(o);
  lp_batch_destroy(h);
  free(ws);
  return 0;
}

static uint64_t mix64(uint64_t x) {  // splitmix64 finaliser: a fixed hash
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}
static double unit(uint64_t a, uint64_t b) { return (mix64(a * 1000003ull + b) >> 11) * 0x1p-53; }

static bool sparse_entry(int pattern, int m, int i, int k) {
  if (pattern == 1) return unit(i, k) < 0.5;
  const int longrow = m > 2150 ? 2150 : m / 2;
  if (i == 7) return false;                                 // an empty row
  if (k == 0) return true;                                  // a dense column
  if (k == 1) return false;                                 // an empty column
  if (i == longrow && k >= 2 && k < 302) return true;       // > one metadata chunk
  if (k < 42) return unit(i, k) < 0.1;
  return unit(i, k) < 0.002;
}

static int sp_flags(long m, long n, const std::vector<int64_t>& rp, const std::vector<int>& ci,
                    const std::vector<double>& v) {
  int flags = 0;
  const long nnz = (long)ci.size();
  pdas::launch_sp_check(nullptr, m, n, nnz, rp.data(), ci.data(), v.data(), &flags);
  return flags;
}

static int run_sparse(int m, int n, int pattern) {
  std::vector<int64_t> rp(m + 1, 0);
  std::vector<int> ci;
  std::vector<double> v;
  for (int i = 0; i < m; ++i) {
    for (int k = 0; k < n; ++k)
      if (sparse_entry(pattern, m, i, k)) {
        ci.push_back(k);
        v.push_back(2.0 * unit(i + 77, k) - 1.0);
      }
    rp[i + 1] = (int64_t)ci.size();
  }
  const long nnz = (long)ci.size();
  const int flags = sp_flags(m, n, rp, ci, v);
  std::vector<int> cnt(n), cur(n), ri(nnz + 1), src(nnz + 1), map(nnz + 1);
  std::vector<int64_t> cp(n + 1, -1);
  std::vector<double> cv(nnz + 1);
  pdas::launch_sp_transpose(nullptr, m, n, nnz, rp.data(), ci.data(), v.data(), cnt.data(),
                            cur.data(), cp.data(), ri.data(), cv.data(), src.data(), map.data());
  // CSC: column counts, rows increasing, values and the CSR -> CSC map
  int csc_bad = 0;
  std::vector<int64_t> colcount(n + 1, 0);
  for (long e = 0; e < nnz; ++e) colcount[ci[e] + 1]++;
  for (int k = 0; k < n; ++k) colcount[k + 1] += colcount[k];
  for (int k = 0; k <= n; ++k) csc_bad += cp[k] != colcount[k];
  for (int k = 0; k < n && !csc_bad; ++k)
    for (int64_t p = cp[k] + 1; p < cp[k + 1]; ++p) csc_bad += ri[p] <= ri[p - 1];
  for (int i = 0; i < m; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int p = map[e];
      csc_bad += !(p >= cp[ci[e]] && p < cp[ci[e] + 1]) || ri[p] != i || cv[p] != v[e];
    }
  // products
  std::vector<double> w(n), d(n), base(m), u1(m), u2(m), out(m, NAN), g1(n, NAN), g2(n, NAN);
  for (int k = 0; k < n; ++k) {
    w[k] = std::sin(0.37 * k + 0.1);
    d[k] = 0.25 + unit(k, 991);
  }
  for (int i = 0; i < m; ++i) {
    base[i] = std::cos(0.11 * i);
    u1[i] = std::sin(0.23 * i + 0.7);
    u2[i] = std::cos(0.19 * i + 0.2);
  }
  pdas::launch_sp_gemv_n(nullptr, m, nnz, rp.data(), ci.data(), v.data(), w.data(), base.data(),
                         out.data(), -1.0);
  pdas::launch_sp_gemv_t(nullptr, n, nnz, cp.data(), ri.data(), cv.data(), u1.data(), u2.data(),
                         g1.data(), g2.data());
  double en = 0, sn = 0, et = 0, st = 0;
  for (int i = 0; i < m; ++i) {
    long double r = 0, a = 0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      r += (long double)v[e] * w[ci[e]];
      a += std::fabs(v[e] * w[ci[e]]);
    }
    en = worse(en, std::fabs((double)(out[i] - (base[i] - r))));
    sn = std::fmax(sn, (double)a + std::fabs(base[i]));
  }
  std::vector<long double> t1(n, 0), t2(n, 0), ta(n, 0);
  for (int i = 0; i < m; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      t1[ci[e]] += (long double)v[e] * u1[i];
      t2[ci[e]] += (long double)v[e] * u2[i];
      ta[ci[e]] += std::fabs(v[e]);
    }
  for (int k = 0; k < n; ++k) {
    et = worse(et, std::fabs((double)(g1[k] - t1[k])));
    et = worse(et, std::fabs((double)(g2[k] - t2[k])));
    st = std::fmax(st, (double)ta[k]);
  }
  // normal matrix: reference summed over the CSC in long double
  const long ldm = m + 3;
  std::vector<double> M((size_t)m * ldm, NAN);
  pdas::launch_sp_syrk(nullptr, m, rp.data(), ci.data(), v.data(), cp.data(), ri.data(),
                       cv.data(), map.data(), d.data(), M.data(), ldm);
  double em = 0, sm = 0;
  int upper_touched = 0;
  std::vector<long double> acc(m);
  for (int i = 0; i < m; ++i) {
    std::fill(acc.begin(), acc.end(), 0.0L);
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int k = ci[e];
      for (int64_t p = colcount[k]; p < colcount[k + 1]; ++p)
        if (ri[p] <= i) acc[ri[p]] += (long double)d[k] * v[e] * cv[p];
    }
    for (int j = 0; j <= i; ++j) {
      em = worse(em, std::fabs((double)(M[(size_t)i * ldm + j] - acc[j])));
      sm = std::fmax(sm, std::fabs((double)acc[j]));
    }
    for (int j = i + 1; j < ldm; ++j) upper_touched += !std::isnan(M[(size_t)i * ldm + j]);
  }
  // the check on broken copies: unsorted row, column out of range, NaN,
  // row_ptr[m] != nnz, a decreasing row_ptr
  int longrow = 0;
  for (int i = 0; i < m; ++i)
    if (rp[i + 1] - rp[i] > rp[longrow + 1] - rp[longrow]) longrow = i;
  auto ci2 = ci;
  std::swap(ci2[rp[longrow]], ci2[rp[longrow] + 1]);
  const int f_unsorted = sp_flags(m, n, rp, ci2, v);
  ci2 = ci;
  ci2[nnz - 1] = n;
  const int f_range = sp_flags(m, n, rp, ci2, v);
  auto v2 = v;
  v2[nnz / 2] = NAN;
  const int f_nan = sp_flags(m, n, rp, ci, v2);
  auto rp2 = rp;
  rp2[m] = nnz - 1;
  std::vector<int> ci3(ci.begin(), ci.end() - 1);
  std::vector<double> v3(v.begin(), v.end() - 1);
  rp2[m] = nnz;  // row_ptr says nnz, the arrays hold nnz - 1: rp[m] != nnz of the call
  const int f_count = sp_flags(m, n, rp2, ci3, v3);
  rp2 = rp;
  rp2[longrow + 1] = rp[longrow] - 1;
  const int f_order = sp_flags(m, n, rp2, ci, v);
  printf("{\"m\": %d, \"n\": %d, \"nnz\": %ld, \"flags\": %d, \"csc_bad\": %d, "
         "\"gemv_n_rel_err\": %.3e, \"gemv_t_rel_err\": %.3e, \"syrk_rel_err\": %.3e, "
         "\"upper_touched\": %d, \"f_unsorted\": %d, \"f_range\": %d, \"f_nan\": %d, "
         "\"f_count\": %d, \"f_order\": %d}\n",
         m, n, nnz, flags, csc_bad, en / sn, et / st, em / sm, upper_touched, f_unsorted,
         f_range, f_nan, f_count, f_order);
  return 0;
}

int main(int argc, char** argv) {
  if (argc >= 3 && !strcmp(argv[1], "chol"))
    return run_chol(atoi(argv[2]), argc >= 4 ? atoi(argv[3]) : 0);
  if (argc >= 6 && !strcmp(argv[1], "syrk"))
    return run_syrk(atoi(argv[2]), atoi(argv[3]), atoi(argv[4]), atoi(argv[5]));
  if (argc >= 3 && !strcmp(argv[1], "trsv")) return run_trsv(atoi(argv[2]));
  if (argc >= 5 && !strcmp(argv[1], "sparse"))
    return run_sparse(atoi(argv[2]), atoi(argv[3]), atoi(argv[4]));
  if (argc >= 6 && !strcmp(argv[1], "batch"))
    return run_batch(argv[2], argv[3], atoi(argv[4]), atoi(argv[5]), argc >= 7 ? atoi(argv[6]) : 0,
                     argc >= 8 ? atoi(argv[7]) : 0);
  fprintf(stderr, "usage: emu chol <m> [g] | emu batch <in> <out> <max_iter> <tape>\n");
  return 1;
}
