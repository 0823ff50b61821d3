"""Each plausible mistake planted in a copy of the oracle source (a dropped
term, a wrong sign, a wrong index, a transposed operand) must make at least
one pin in tests/pins.py fail.  Mutants are compiled on the CPU into a
temporary directory; the real oracle is never modified."""
import os
import subprocess

import pytest

import pins
from oracle import build as obuild

MUTANTS = {
    "ds_sign": ("S->ds[j] = S->rd[j] - S->g[j];", "S->ds[j] = S->rd[j] + S->g[j];"),
    "rhs_dropped_term": ("S->rhs[i] = S->b[i] + S->rhs[i];", "S->rhs[i] = S->b[i];"),
    "d_inverted": ("S->d[j] = S->x[j] / S->s[j];", "S->d[j] = S->s[j] / S->x[j];"),
    "normal_wrong_index": ("acc += A[i * n + j] * d[j] * A[k * n + j];",
                           "acc += A[i * n + j] * d[i] * A[k * n + j];"),
    "ratio_wrong_vector": ("real u = -S->dx[j] / S->x[j];", "real u = -S->dx[j] / S->s[j];"),
    "step_length": ("real t = aeff / psi;", "real t = aeff * psi;"),
    "cholesky_index": ("for (long k = 0; k < j; ++k) acc -= L[i * m + k] * L[j * m + k];",
                       "for (long k = 0; k < j; ++k) acc -= L[i * m + k] * L[i * m + k];"),
    "backsolve_transposed": ("for (long k = i + 1; k < m; ++k) acc -= L[k * m + i] * w[k];",
                             "for (long k = i + 1; k < m; ++k) acc -= L[i * m + k] * w[k];"),
    "rd_sign": ("S->rd[j] = S->c[j] - S->g[j] - S->s[j];",
                "S->rd[j] = S->c[j] - S->g[j] + S->s[j];"),
    "argmax_block": ("if (v > psi) { psi = v; arg = n + j; }", "if (v > psi) { psi = v; arg = j; }"),
    "adjoint_sign": ("for (long i = 0; i < m; ++i) dyb[i] -= tmpm[i];",
                     "for (long i = 0; i < m; ++i) dyb[i] += tmpm[i];"),
    "adjoint_dropped_term": ("for (long j = 0; j < n; ++j) db_[j] -= h[j] * g[j];", ""),
    "adjoint_abar_transposed": ("lam[i] * S.d[j] * S.rd[j] - y[i] * rdb[j];",
                                "lam[i] * S.d[j] * S.rd[j] - y[i] * dsb[j];"),
    "jvp_sign": ("for (long j = 0; j < n; ++j) Tds[j] = Trd[j] - Tg[j];",
                 "for (long j = 0; j < n; ++j) Tds[j] = Trd[j] + Tg[j];"),
    "psi1_rule": ("real aeff = (psi == 1) ? (real)1 : alpha;", "real aeff = alpha;"),
    "pc_corrector_term": ("rc[j] = -S->x[j] * S->s[j] - dxa[j] * dsa[j] + info->sigma * info->mu;",
                          "rc[j] = -S->x[j] * S->s[j] + info->sigma * info->mu;"),
    "pc_rhs_sign": ("t[j] = S->d[j] * S->rd[j] - S->x[j] - rc[j] / S->s[j];",
                    "t[j] = S->d[j] * S->rd[j] - S->x[j] + rc[j] / S->s[j];"),
    "pc_dual_step_on_x": ("S->x[j] = S->x[j] + info->a_p * S->dx[j];",
                          "S->x[j] = S->x[j] + info->a_d * S->dx[j];"),
    "pc_no_centring": ("rc[j] = -S->x[j] * S->s[j] - dxa[j] * dsa[j] + info->sigma * info->mu;",
                       "rc[j] = -S->x[j] * S->s[j] - dxa[j] * dsa[j];"),
    "pc_eta_dropped": ("info->a_p = eta * mp < 1 ? eta * mp : (real)1;",
                       "info->a_p = mp < 1 ? mp : (real)1;"),
}


def _build_mutant(tmpdir, name, old, new):
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path_c = os.path.join(tmpdir, f"mut_{name}.c")
    path_so = os.path.join(tmpdir, f"libmut_{name}.so")
    open(path_c, "w").write(src.replace(old, new))
    subprocess.run(["gcc", "-std=gnu99", "-O2", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-w", "-DREAL=double", path_c, "-o", path_so, "-lm"],
                   check=True)
    return path_so


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    lib = _build_mutant(str(tmp_path), name, old, new)
    caught = []
    for check in pins.ALL_CHECKS:
        try:
            check(lib)
        except Exception as e:  # assertion or numerical blow-up both count
            caught.append((check.__name__, type(e).__name__))
    assert caught, f"mutant {name} passed every pin"
