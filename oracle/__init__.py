"""CPU oracle for Primal-Dual Affine Scaling -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The GPU library and its Python
binding never import it; the two implementations share no code.

This module is a thin ctypes wrapper over ``pdas_oracle.c`` (plain C loops in
double or long double, written from the paper's Section 3 algorithm and its
Section 5 reduction to the normal equations).  All arrays are numpy float64,
A row-major (m, n).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

# Status numbering of the oracle library (its own).
CONTINUE = 0
CONVERGED = 1
OPTIMAL_PSI1 = 2
OPTIMAL_ZERO_DIR = 3
MAX_ITER = 4
ERR_INVALID_ARG = -1
ERR_SHAPE = -2
ERR_NOT_INTERIOR = -3
ERR_BREAKDOWN = -4
ERR_NONPOS_PSI = -5
ERR_LOST_INTERIOR = -6

STATUS_NAMES = {
    CONTINUE: "CONTINUE", CONVERGED: "CONVERGED", OPTIMAL_PSI1: "OPTIMAL_PSI1",
    OPTIMAL_ZERO_DIR: "OPTIMAL_ZERO_DIR", MAX_ITER: "MAX_ITER",
    ERR_INVALID_ARG: "ERR_INVALID_ARG", ERR_SHAPE: "ERR_SHAPE",
    ERR_NOT_INTERIOR: "ERR_NOT_INTERIOR", ERR_BREAKDOWN: "ERR_BREAKDOWN",
    ERR_NONPOS_PSI: "ERR_NONPOS_PSI", ERR_LOST_INTERIOR: "ERR_LOST_INTERIOR",
}

_dp = C.POINTER(C.c_double)


class _IterOut(C.Structure):
    _fields_ = [
        ("r_d", _dp), ("r_p", _dp), ("d", _dp), ("M", _dp), ("L", _dp), ("rhs", _dp),
        ("dx", _dp), ("dy", _dp), ("ds", _dp),
        ("gap", C.c_double), ("psi", C.c_double), ("t", C.c_double),
        ("alpha_eff", C.c_double), ("argmax", C.c_longlong), ("min_pivot", C.c_double),
        ("fail_col", C.c_longlong),
    ]


class _Log(C.Structure):
    _fields_ = [
        ("gap", C.c_double), ("psi", C.c_double), ("t", C.c_double),
        ("argmax", C.c_longlong), ("rp_norm", C.c_double), ("rd_norm", C.c_double),
        ("min_pivot", C.c_double),
    ]


class _PCOut(C.Structure):
    _fields_ = [
        ("dx_aff", _dp), ("dy_aff", _dp), ("ds_aff", _dp), ("dx", _dp), ("dy", _dp),
        ("ds", _dp), ("rhs_aff", _dp), ("rhs", _dp),
        ("gap", C.c_double), ("mu", C.c_double), ("mu_aff", C.c_double), ("sigma", C.c_double),
        ("alpha_aff_p", C.c_double), ("alpha_aff_d", C.c_double), ("alpha_p", C.c_double),
        ("alpha_d", C.c_double), ("min_pivot", C.c_double), ("fail_col", C.c_longlong),
    ]


class _PCLog(C.Structure):
    _fields_ = [("gap", C.c_double), ("sigma", C.c_double), ("alpha_p", C.c_double),
                ("alpha_d", C.c_double), ("min_pivot", C.c_double)]


_libs: dict = {}


def _bind(lib):
    L, I, D, P = C.c_long, C.c_int, C.c_double, _dp
    lib.orc_iterate.argtypes = [L, L, P, P, P, P, P, P, D, C.POINTER(_IterOut)]
    lib.orc_iterate.restype = I
    lib.orc_solve.argtypes = [L, L, P, P, P, P, P, P, D, D, I, C.POINTER(I),
                              C.POINTER(_Log), P]
    lib.orc_solve.restype = I
    lib.orc_forward_k.argtypes = [L, L, P, P, P, P, P, P, D, I, P, P, P, P, P, P, D, P,
                                  P, P, P, P]
    lib.orc_forward_k.restype = I
    lib.orc_backward.argtypes = [L, L, P, P, P, D, I, P, P, P, P, P, P, P, P, P, P]
    lib.orc_backward.restype = I
    lib.orc_jvp.argtypes = [L, L, P, P, P, P, P, P, D, I, P, P, P, P, P, P, P, P, P]
    lib.orc_jvp.restype = I
    lib.orc_normal_matrix.argtypes = [L, L, P, P, P]
    lib.orc_normal_matrix.restype = None
    lib.orc_cholesky.argtypes = [L, P, P, P]
    lib.orc_cholesky.restype = C.c_long
    lib.orc_cholesky_solve.argtypes = [L, P, P, P]
    lib.orc_cholesky_solve.restype = None
    lib.orc_pc_iterate.argtypes = [L, L, P, P, P, P, P, P, D, C.POINTER(_PCOut)]
    lib.orc_pc_iterate.restype = I
    lib.orc_pc_solve.argtypes = [L, L, P, P, P, P, P, P, D, D, I, C.POINTER(I),
                                 C.POINTER(_PCLog)]
    lib.orc_pc_solve.restype = I
    lib.orc_num_threads.restype = I
    lib.orc_real_bytes.restype = I
    return lib


def _lib(precision: str = "f64"):
    """The oracle library for ``precision`` ('f64' or 'f80'), or a path to a
    library built from a (test-modified) copy of the same source."""
    if precision not in _libs:
        if precision in _build.VARIANTS:
            _build.ensure_built()
            path = _build.lib_path(precision)
        else:
            path = precision
        _libs[precision] = _bind(C.CDLL(path))
    return _libs[precision]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def num_threads() -> int:
    return _lib().orc_num_threads()


@dataclass
class IterResult:
    status: int
    x: np.ndarray
    y: np.ndarray
    s: np.ndarray
    r_d: np.ndarray
    r_p: np.ndarray
    d: np.ndarray
    M: np.ndarray
    L: np.ndarray
    rhs: np.ndarray
    dx: np.ndarray
    dy: np.ndarray
    ds: np.ndarray
    gap: float
    psi: float
    t: float
    alpha_eff: float
    argmax: int
    min_pivot: float
    fail_col: int

    @property
    def status_name(self) -> str:
        return STATUS_NAMES[self.status]


def iterate(A, b, c, x, y, s, alpha, precision="f64") -> IterResult:
    """One pass of the Algorithm's loop body from (x, y, s)."""
    A, b, c = _f64(A), _f64(b), _f64(c)
    x, y, s = _f64(x).copy(), _f64(y).copy(), _f64(s).copy()
    m, n = A.shape
    bufs = {k: np.full(sz, np.nan) for k, sz in
            dict(r_d=n, r_p=m, d=n, M=(m, m), L=(m, m), rhs=m, dx=n, dy=m, ds=n).items()}
    out = _IterOut(**{k: _p(v) for k, v in bufs.items()})
    st = _lib(precision).orc_iterate(m, n, _p(A), _p(b), _p(c), _p(x), _p(y), _p(s),
                                     float(alpha), C.byref(out))
    return IterResult(status=st, x=x, y=y, s=s, gap=out.gap, psi=out.psi, t=out.t,
                      alpha_eff=out.alpha_eff, argmax=out.argmax, min_pivot=out.min_pivot,
                      fail_col=out.fail_col, **bufs)


@dataclass
class SolveResult:
    status: int
    iters: int
    x: np.ndarray
    y: np.ndarray
    s: np.ndarray
    log: list = field(default_factory=list)
    tape: np.ndarray | None = None

    @property
    def status_name(self) -> str:
        return STATUS_NAMES[self.status]


def solve(A, b, c, x0, y0, s0, alpha=0.95, gap_tol=1e-8, max_iter=200, tape=False,
          precision="f64") -> SolveResult:
    """The Algorithm's loop, stopping on x^T s < gap_tol or after max_iter steps."""
    A, b, c = _f64(A), _f64(b), _f64(c)
    x, y, s = _f64(x0).copy(), _f64(y0).copy(), _f64(s0).copy()
    m, n = A.shape
    logs = (_Log * max(max_iter, 1))()
    tp = np.zeros((max_iter + 1, 2 * n + m)) if tape else None
    iters = C.c_int(0)
    st = _lib(precision).orc_solve(m, n, _p(A), _p(b), _p(c), _p(x), _p(y), _p(s),
                                   float(alpha), float(gap_tol), int(max_iter),
                                   C.byref(iters), logs, _p(tp))
    k = iters.value
    # a step that ended in an error or the zero-direction stop was logged too
    nlog = min(k + (1 if st in (ERR_BREAKDOWN, ERR_NONPOS_PSI, ERR_LOST_INTERIOR,
                                OPTIMAL_ZERO_DIR) else 0), max_iter)
    log = [dict(gap=logs[i].gap, psi=logs[i].psi, t=logs[i].t, argmax=logs[i].argmax,
                rp_norm=logs[i].rp_norm, rd_norm=logs[i].rd_norm,
                min_pivot=logs[i].min_pivot) for i in range(nlog)]
    return SolveResult(status=st, iters=k, x=x, y=y, s=s, log=log,
                       tape=None if tp is None else tp[: k + 1].copy())


def forward_k(A, b, c, x0, y0, s0, alpha, K, w, direction=None, h=0.0, precision="f64"):
    """Exactly K steps from the start (A,b,c,x0,y0,s0) + h*direction, formed in the
    oracle's REAL precision.  Returns (status, w^T x_K, x_K, y_K, s_K)."""
    A, b, c = _f64(A), _f64(b), _f64(c)
    x0, y0, s0, w = _f64(x0), _f64(y0), _f64(s0), _f64(w)
    m, n = A.shape
    dirs = dict(A=None, b=None, c=None, x0=None, y0=None, s0=None)
    if direction:
        for k, v in direction.items():
            dirs[k] = _f64(v)
    loss = C.c_double(np.nan)
    xK, yK, sK = np.zeros(n), np.zeros(m), np.zeros(n)
    st = _lib(precision).orc_forward_k(
        m, n, _p(A), _p(b), _p(c), _p(x0), _p(y0), _p(s0), float(alpha), int(K),
        _p(dirs["A"]), _p(dirs["b"]), _p(dirs["c"]), _p(dirs["x0"]), _p(dirs["y0"]),
        _p(dirs["s0"]), float(h), _p(w), C.byref(loss), _p(xK), _p(yK), _p(sK))
    return st, loss.value, xK, yK, sK


def backward(A, b, c, alpha, K, tape, xbar, ybar=None, sbar=None, precision="f64"):
    """Reverse mode through the K steps recorded in ``tape`` (rows of [x|y|s]).
    Returns (status, dict of Abar, bbar, cbar, x0bar, y0bar, s0bar)."""
    A, b, c, tape = _f64(A), _f64(b), _f64(c), _f64(tape)
    m, n = A.shape
    xbar = _f64(xbar)
    ybar = None if ybar is None else _f64(ybar)
    sbar = None if sbar is None else _f64(sbar)
    out = dict(Abar=np.zeros((m, n)), bbar=np.zeros(m), cbar=np.zeros(n),
               x0bar=np.zeros(n), y0bar=np.zeros(m), s0bar=np.zeros(n))
    st = _lib(precision).orc_backward(
        m, n, _p(A), _p(b), _p(c), float(alpha), int(K), _p(tape), _p(xbar), _p(ybar),
        _p(sbar), _p(out["Abar"]), _p(out["bbar"]), _p(out["cbar"]), _p(out["x0bar"]),
        _p(out["y0bar"]), _p(out["s0bar"]))
    return st, out


def jvp(A, b, c, x0, y0, s0, alpha, K, tangents, precision="f64"):
    """Forward-mode tangents of (x_K, y_K, s_K) for input tangents
    (dict with any of A, b, c, x0, y0, s0)."""
    A, b, c = _f64(A), _f64(b), _f64(c)
    x0, y0, s0 = _f64(x0), _f64(y0), _f64(s0)
    m, n = A.shape
    t = {k: None for k in ("A", "b", "c", "x0", "y0", "s0")}
    for k, v in tangents.items():
        t[k] = _f64(v)
    tx, ty, ts = np.zeros(n), np.zeros(m), np.zeros(n)
    st = _lib(precision).orc_jvp(
        m, n, _p(A), _p(b), _p(c), _p(x0), _p(y0), _p(s0), float(alpha), int(K),
        _p(t["A"]), _p(t["b"]), _p(t["c"]), _p(t["x0"]), _p(t["y0"]), _p(t["s0"]),
        _p(tx), _p(ty), _p(ts))
    return st, tx, ty, ts


def normal_matrix(A, d, precision="f64"):
    A, d = _f64(A), _f64(d)
    m, n = A.shape
    M = np.zeros((m, m))
    _lib(precision).orc_normal_matrix(m, n, _p(A), _p(d), _p(M))
    return M


def cholesky(M, precision="f64"):
    """Returns (L, fail_col, min_pivot); fail_col = -1 on success."""
    M = _f64(M)
    m = M.shape[0]
    L = np.zeros((m, m))
    mp = C.c_double(np.nan)
    f = _lib(precision).orc_cholesky(m, _p(M), _p(L), C.byref(mp))
    return L, int(f), mp.value


def cholesky_solve(L, r, precision="f64"):
    L, r = _f64(L), _f64(r)
    m = L.shape[0]
    w = np.zeros(m)
    _lib(precision).orc_cholesky_solve(m, _p(L), _p(r), _p(w))
    return w


@dataclass
class PCResult:
    status: int
    x: np.ndarray
    y: np.ndarray
    s: np.ndarray
    dx_aff: np.ndarray
    dy_aff: np.ndarray
    ds_aff: np.ndarray
    dx: np.ndarray
    dy: np.ndarray
    ds: np.ndarray
    rhs_aff: np.ndarray
    rhs: np.ndarray
    gap: float
    mu: float
    mu_aff: float
    sigma: float
    alpha_aff_p: float
    alpha_aff_d: float
    alpha_p: float
    alpha_d: float
    min_pivot: float
    fail_col: int

    @property
    def status_name(self) -> str:
        return STATUS_NAMES[self.status]


def pc_iterate(A, b, c, x, y, s, eta=0.95, precision="f64") -> PCResult:
    """One predictor-corrector (Mehrotra) iteration from (x, y, s)."""
    A, b, c = _f64(A), _f64(b), _f64(c)
    x, y, s = _f64(x).copy(), _f64(y).copy(), _f64(s).copy()
    m, n = A.shape
    bufs = {k: np.full(sz, np.nan) for k, sz in
            dict(dx_aff=n, dy_aff=m, ds_aff=n, dx=n, dy=m, ds=n, rhs_aff=m, rhs=m).items()}
    out = _PCOut(**{k: _p(v) for k, v in bufs.items()})
    st = _lib(precision).orc_pc_iterate(m, n, _p(A), _p(b), _p(c), _p(x), _p(y), _p(s),
                                        float(eta), C.byref(out))
    sc = {k: getattr(out, k) for k in ("gap", "mu", "mu_aff", "sigma", "alpha_aff_p",
                                      "alpha_aff_d", "alpha_p", "alpha_d", "min_pivot")}
    return PCResult(status=st, x=x, y=y, s=s, fail_col=out.fail_col, **sc, **bufs)


def pc_solve(A, b, c, x0, y0, s0, eta=0.95, gap_tol=1e-8, max_iter=200,
             precision="f64") -> SolveResult:
    """The predictor-corrector loop, stopping on x^T s < gap_tol or after
    max_iter steps; log entries hold gap, sigma, alpha_p, alpha_d, min_pivot."""
    A, b, c = _f64(A), _f64(b), _f64(c)
    x, y, s = _f64(x0).copy(), _f64(y0).copy(), _f64(s0).copy()
    m, n = A.shape
    logs = (_PCLog * max(max_iter, 1))()
    iters = C.c_int(0)
    st = _lib(precision).orc_pc_solve(m, n, _p(A), _p(b), _p(c), _p(x), _p(y), _p(s),
                                      float(eta), float(gap_tol), int(max_iter),
                                      C.byref(iters), logs)
    k = iters.value
    nlog = min(k + (1 if st in (ERR_BREAKDOWN, ERR_NONPOS_PSI, ERR_LOST_INTERIOR,
                                OPTIMAL_ZERO_DIR) else 0), max_iter)
    log = [dict(gap=logs[i].gap, sigma=logs[i].sigma, alpha_p=logs[i].alpha_p,
                alpha_d=logs[i].alpha_d, min_pivot=logs[i].min_pivot) for i in range(nlog)]
    return SolveResult(status=st, iters=k, x=x, y=y, s=s, log=log)
