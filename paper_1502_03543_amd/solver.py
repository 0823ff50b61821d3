"""PyTorch-facing wrappers over the libpdas C ABI.

PyTorch provides device memory (the workspace and the vectors) and the
stream (``torch.cuda.current_stream()``); every computation happens in the
library's HIP kernels.  Tensors must be float64, contiguous, on a ROCm GPU.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import capi

_PREC = {"fp64": capi.LP_PREC_FP64, "mixed": capi.LP_PREC_MIXED}
_METHOD = {"affine": capi.LP_METHOD_AFFINE, "pc": capi.LP_METHOD_PC}
_SOLVER = {"cholesky": capi.LP_SOLVER_CHOLESKY, "woodbury": capi.LP_SOLVER_WOODBURY}


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (ROCm) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def workspace(nbytes: int, device) -> tuple[torch.Tensor, int]:
    """A device byte buffer and a 256-byte aligned address inside it."""
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    addr = (buf.data_ptr() + 255) // 256 * 256
    return buf, addr


def options(alpha=0.95, precision="fp64", tape_capacity=0, mixed_switch_gap=1e-6,
            refine_tol=2.0 ** -46, refine_max=5, profile=False, syrk_tile=0, syrk_splits=0,
            syrk32_splits=0, method="affine", solver="cholesky", batch_tile=0,
            batch_graph_iters=0) -> capi.lp_options:
    o = capi.lp_options()
    capi.lp_options_default(C.byref(o))
    o.alpha = float(alpha)
    o.precision = _PREC[precision]
    o.tape_capacity = int(tape_capacity)
    o.mixed_switch_gap = float(mixed_switch_gap)
    o.refine_tol = float(refine_tol)
    o.refine_max = int(refine_max)
    # True (or 1): every phase; "kernel" (or 2): the normal-matrix kernel alone
    o.profile = 2 if profile in ("kernel", 2) else int(bool(profile))
    o.syrk_tile = int(syrk_tile)
    o.syrk_splits = int(syrk_splits)
    o.syrk32_splits = int(syrk32_splits)
    o.method = _METHOD[method]
    o.solver = _SOLVER[solver]
    o.batch_tile = int(batch_tile)
    o.batch_graph_iters = int(batch_graph_iters)
    return o


def tuned_launch(precision: str, m: int, n: int) -> dict:
    """Normal-matrix launch choices measured by the autotuner for this shape
    (empty when none are cached: the library then chooses)."""
    from . import autotune

    out = {}
    e64 = autotune.lookup("fp64", m, n)
    if e64:
        out.update({k: e64["choice"][k] for k in ("syrk_tile", "syrk_splits")})
    if precision == "mixed":
        e32 = autotune.lookup("mixed", m, n)
        if e32:
            out["syrk32_splits"] = e32["choice"]["syrk32_splits"]
    return out


def tuned_batch_launch(m, n) -> dict:
    """Batched launch choices (tile, iterations per graph) measured by the
    autotuner for a batch of this shape signature (empty when none)."""
    from . import autotune

    e = autotune.lookup_batch(m, n)
    return dict(e["choice"]) if e else {}


class LP:
    """One LP on the GPU (lp_setup ... lp_destroy)."""

    def __init__(self, A, b, c, x0, y0, s0, **opts):
        m, n = A.shape
        for t, shp, nm in ((A, (m, n), "A"), (b, (m,), "b"), (c, (n,), "c"), (x0, (n,), "x0"),
                           (y0, (m,), "y0"), (s0, (n,), "s0")):
            _need(t, shp, nm)
        self.m, self.n = m, n
        self.device = A.device
        if not any(k in opts for k in ("syrk_tile", "syrk_splits", "syrk32_splits")):
            opts.update(tuned_launch(opts.get("precision", "fp64"), m, n))
        self.opts = options(**opts)
        size = C.c_size_t(0)
        capi.check(capi.lp_workspace_size(m, n, C.byref(self.opts), C.byref(size)),
                   "lp_workspace_size")
        self._ws, addr = workspace(size.value, A.device)
        self._A = A  # borrowed by the handle
        h = C.c_void_p()
        st = capi.lp_setup(C.byref(h), m, n, _p(A), _p(b), _p(c), _p(x0), _p(y0), _p(s0),
                           C.byref(self.opts), C.c_void_p(addr), size.value, _stream())
        capi.check(st, "lp_setup")
        self.h = h

    def iterate(self) -> dict:
        info = capi.lp_iter_info()
        st = capi.lp_iterate(self.h, C.byref(info))
        d = info.as_dict()
        d["status"] = st
        return d

    def solve(self, tol=1e-8, max_iter=500, want_log=False):
        res = capi.lp_result()
        log = (capi.lp_iter_info * max(1, max_iter))() if want_log else None
        st = capi.lp_solve(self.h, float(tol), int(max_iter), C.byref(res), log)
        out = dict(status=st, iters=res.iters, gap=res.gap, primal_obj=res.primal_obj,
                   dual_obj=res.dual_obj)
        if want_log:
            out["log"] = [log[i].as_dict() for i in range(min(res.iters + (1 if st < 0 else 0),
                                                                max_iter))]
        return out

    def iterate_values(self):
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        y = torch.empty(self.m, dtype=torch.float64, device=self.device)
        s = torch.empty(self.n, dtype=torch.float64, device=self.device)
        capi.check(capi.lp_get_iterate(self.h, _p(x), _p(y), _p(s)), "lp_get_iterate")
        return x, y, s

    def tape(self, K):
        """The first K recorded start iterates as a (K, 2n + m) numpy array of
        rows [x | y | s]."""
        import numpy as np
        rows = []
        for k in range(K):
            x = torch.empty(self.n, dtype=torch.float64, device=self.device)
            y = torch.empty(self.m, dtype=torch.float64, device=self.device)
            s = torch.empty(self.n, dtype=torch.float64, device=self.device)
            capi.check(capi.lp_tape_row(self.h, k, _p(x), _p(y), _p(s)), "lp_tape_row")
            rows.append(torch.cat([x, y, s]).cpu().numpy())
        return np.stack(rows)

    def direction(self):
        """(dx, dy, ds) of the most recent iterate() call."""
        dx = torch.empty(self.n, dtype=torch.float64, device=self.device)
        dy = torch.empty(self.m, dtype=torch.float64, device=self.device)
        ds = torch.empty(self.n, dtype=torch.float64, device=self.device)
        capi.check(capi.lp_get_direction(self.h, _p(dx), _p(dy), _p(ds)), "lp_get_direction")
        return dx, dy, ds

    def timings(self) -> dict:
        t = capi.lp_timings()
        capi.check(capi.lp_get_timings(self.h, C.byref(t)), "lp_get_timings")
        return t.as_dict()

    def close(self):
        if getattr(self, "h", None):
            capi.lp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _need_csr(row_ptr, col_idx, vals, m):
    if not all(isinstance(t, torch.Tensor) and t.device.type == "cuda" and t.is_contiguous()
               for t in (row_ptr, col_idx, vals)):
        raise TypeError("row_ptr, col_idx and vals must be contiguous CUDA (ROCm) tensors")
    if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32 or vals.dtype != torch.float64:
        raise TypeError("row_ptr int64, col_idx int32 and vals float64 are required")
    if row_ptr.shape != (m + 1,) or col_idx.dim() != 1 or vals.shape != col_idx.shape:
        raise ValueError("row_ptr must have m + 1 entries and col_idx, vals nnz each")
    return int(col_idx.shape[0])


class CsrLP(LP):
    """One LP whose A is given in canonical CSR (lp_setup_csr): row_ptr
    (int64, m + 1), col_idx (int32, nnz, strictly increasing per row), vals
    (float64, nnz), all borrowed for the handle's lifetime."""

    def __init__(self, row_ptr, col_idx, vals, shape, b, c, x0, y0, s0, **opts):
        m, n = (int(v) for v in shape)
        nnz = _need_csr(row_ptr, col_idx, vals, m)
        for t, shp, nm in ((b, (m,), "b"), (c, (n,), "c"), (x0, (n,), "x0"), (y0, (m,), "y0"),
                           (s0, (n,), "s0")):
            _need(t, shp, nm)
        self.m, self.n, self.nnz = m, n, nnz
        self.device = b.device
        self.opts = options(**opts)
        size = C.c_size_t(0)
        capi.check(capi.lp_workspace_size_csr(m, n, nnz, C.byref(self.opts), C.byref(size)),
                   "lp_workspace_size_csr")
        self._ws, addr = workspace(size.value, b.device)
        self._A = (row_ptr, col_idx, vals)  # borrowed by the handle
        h = C.c_void_p()
        st = capi.lp_setup_csr(C.byref(h), m, n, nnz, _p(row_ptr), _p(col_idx), _p(vals),
                               _p(b), _p(c), _p(x0), _p(y0), _p(s0), C.byref(self.opts),
                               C.c_void_p(addr), size.value, _stream())
        capi.check(st, "lp_setup_csr")
        self.h = h


def normal_matrix_csr(row_ptr, col_idx, vals, shape, d):
    """Lower triangle of A diag(d) A^T for A in canonical CSR (upper zero)."""
    m, n = (int(v) for v in shape)
    nnz = _need_csr(row_ptr, col_idx, vals, m)
    _need(d, (n,), "d")
    M = torch.zeros((m, m), dtype=torch.float64, device=d.device)
    size = C.c_size_t(0)
    capi.check(capi.lp_csr_workspace_size(m, n, nnz, C.byref(size)), "lp_csr_workspace_size")
    buf, addr = workspace(size.value, d.device)
    capi.check(capi.lp_normal_matrix_csr(m, n, nnz, _p(row_ptr), _p(col_idx), _p(vals), _p(d),
                                         _p(M), m, C.c_void_p(addr), size.value, _stream()),
               "lp_normal_matrix_csr")
    torch.cuda.current_stream().synchronize()
    return M


def solve(A, b, c, x0, y0, s0, alpha=0.95, tol=1e-8, max_iter=500, precision="fp64"):
    """Run the Section 3 loop on the GPU.  Returns (x, y, s, info); raises
    RuntimeError (with the status name) on an error status."""
    lp = LP(A, b, c, x0, y0, s0, alpha=alpha, precision=precision)
    info = lp.solve(tol, max_iter)
    capi.check(info["status"], "lp_solve")
    x, y, s = lp.iterate_values()
    torch.cuda.current_stream().synchronize()
    info["status_name"] = capi.status_string(info["status"])
    lp.close()
    return x, y, s, info


def _blocks_ws(m, n, device):
    size = C.c_size_t(0)
    capi.check(capi.lp_blocks_workspace_size(m, n, C.byref(size)), "lp_blocks_workspace_size")
    buf, addr = workspace(size.value, device)
    return buf, addr, size.value


def normal_matrix(A, d):
    """Lower triangle of A diag(d) A^T (upper triangle zero)."""
    m, n = A.shape
    _need(A, (m, n), "A")
    _need(d, (n,), "d")
    M = torch.zeros((m, m), dtype=torch.float64, device=A.device)
    buf, addr, nb = _blocks_ws(m, n, A.device)
    capi.check(capi.lp_normal_matrix(m, n, _p(A), _p(d), _p(M), m, C.c_void_p(addr), nb,
                                     _stream()), "lp_normal_matrix")
    torch.cuda.current_stream().synchronize()
    return M


def cholesky(M):
    """In-place Cholesky of a copy of M's lower triangle.  Returns
    (L, fail_col, min_pivot, status); upper triangle of L zeroed."""
    m = M.shape[0]
    _need(M, (m, m), "M")
    L = M.clone()
    buf, addr, nb = _blocks_ws(m, m + 1, M.device)
    fail = C.c_int64(0)
    minp = C.c_double(0)
    st = capi.lp_cholesky(m, _p(L), m, C.c_void_p(addr), nb, _stream(), C.byref(fail),
                          C.byref(minp))
    if st not in (capi.LP_OK, capi.LP_ERR_BREAKDOWN):
        capi.check(st, "lp_cholesky")
    return torch.tril(L), fail.value, minp.value, st


def chol_solve(L, r):
    m = L.shape[0]
    _need(L, (m, m), "L")
    _need(r, (m,), "r")
    dy = torch.empty_like(r)
    buf, addr, nb = _blocks_ws(m, m + 1, L.device)
    capi.check(capi.lp_chol_solve(m, _p(L), m, _p(r), _p(dy), C.c_void_p(addr), nb, _stream()),
               "lp_chol_solve")
    torch.cuda.current_stream().synchronize()
    return dy


class Batch:
    """Many LPs solved together (lp_batch_setup ... lp_batch_destroy).

    ``problems`` is a list of objects with numpy fields A (m_i x n_i), b, c,
    x0, y0, s0; they are packed on the host, uploaded once, and solved by the
    batched kernels, in FP64 or (precision="mixed") with the FP32 factor and
    FP64 refinement per LP."""

    def __init__(self, problems, alpha=0.95, tape_capacity=0, device="cuda", batch_tile=None,
                 batch_graph_iters=None, precision="fp64", refine_max=5, refine_tol=2.0 ** -46,
                 mixed_switch_gap=1e-6):
        import numpy as np

        self.count = len(problems)
        self.m = np.array([p.A.shape[0] for p in problems], dtype=np.int64)
        self.n = np.array([p.A.shape[1] for p in problems], dtype=np.int64)
        mn = self.m * self.n
        self.a_off = np.concatenate([[0], np.cumsum(mn)[:-1]]).astype(np.int64)
        self.v_off_m = np.concatenate([[0], np.cumsum(self.m)[:-1]]).astype(np.int64)
        self.v_off_n = np.concatenate([[0], np.cumsum(self.n)[:-1]]).astype(np.int64)
        cat = lambda k: np.ascontiguousarray(
            np.concatenate([np.asarray(getattr(p, k), dtype=np.float64).ravel() for p in problems]))
        dev = torch.device(device)
        self.A = torch.from_numpy(cat("A")).to(dev)
        self.b = torch.from_numpy(cat("b")).to(dev)
        self.c = torch.from_numpy(cat("c")).to(dev)
        self.x0 = torch.from_numpy(cat("x0")).to(dev)
        self.y0 = torch.from_numpy(cat("y0")).to(dev)
        self.s0 = torch.from_numpy(cat("s0")).to(dev)
        self.device = dev
        if batch_tile is None and batch_graph_iters is None:
            tuned = tuned_batch_launch(self.m, self.n)
            batch_tile = tuned.get("batch_tile", 0)
            batch_graph_iters = tuned.get("batch_graph_iters", 0)
        self.opts = options(alpha=alpha, tape_capacity=tape_capacity, precision=precision,
                            refine_max=refine_max, refine_tol=refine_tol,
                            mixed_switch_gap=mixed_switch_gap, batch_tile=batch_tile or 0,
                            batch_graph_iters=batch_graph_iters or 0)
        I64 = C.c_int64 * self.count
        self._m, self._n = I64(*self.m), I64(*self.n)
        self._aoff, self._vom, self._von = I64(*self.a_off), I64(*self.v_off_m), I64(*self.v_off_n)
        size = C.c_size_t(0)
        capi.check(capi.lp_batch_workspace_size(self.count, self._m, self._n, C.byref(self.opts),
                                                C.byref(size)), "lp_batch_workspace_size")
        self._ws, addr = workspace(size.value, dev)
        h = C.c_void_p()
        st = capi.lp_batch_setup(C.byref(h), self.count, self._m, self._n, _p(self.A), self._aoff,
                                 _p(self.b), _p(self.c), _p(self.x0), _p(self.y0), _p(self.s0),
                                 self._vom, self._von, C.byref(self.opts), C.c_void_p(addr),
                                 size.value, _stream())
        capi.check(st, "lp_batch_setup")
        self.h = h

    def solve(self, tol=1e-8, max_iter=200):
        import numpy as np

        stat = (C.c_int32 * self.count)()
        its = (C.c_int32 * self.count)()
        nconv = C.c_int32(0)
        capi.check(capi.lp_batch_solve(self.h, float(tol), int(max_iter), stat, its,
                                       C.byref(nconv)), "lp_batch_solve")
        return dict(status=np.array(stat[:]), iters=np.array(its[:]), n_converged=nconv.value)

    def iterate(self, tol=0.0):
        """One loop pass for every running LP (lp_batch_iterate).  Returns
        (status array, list of per-LP step dicts, caller's LP order)."""
        import numpy as np

        stat = (C.c_int32 * self.count)()
        info = (capi.lp_iter_info * self.count)()
        capi.check(capi.lp_batch_iterate(self.h, float(tol), stat, info), "lp_batch_iterate")
        return np.array(stat[:]), [info[i].as_dict() for i in range(self.count)]

    def iterates(self):
        """List of (x, y, s) numpy arrays, one per LP."""
        sn, sm = int(self.n.sum()), int(self.m.sum())
        x = torch.empty(sn, dtype=torch.float64, device=self.device)
        y = torch.empty(sm, dtype=torch.float64, device=self.device)
        s = torch.empty(sn, dtype=torch.float64, device=self.device)
        capi.check(capi.lp_batch_get_iterate(self.h, _p(x), _p(y), _p(s)), "lp_batch_get_iterate")
        torch.cuda.current_stream().synchronize()
        x, y, s = x.cpu().numpy(), y.cpu().numpy(), s.cpu().numpy()
        out = []
        for i in range(self.count):
            jn, jm = self.v_off_n[i], self.v_off_m[i]
            out.append((x[jn:jn + self.n[i]], y[jm:jm + self.m[i]], s[jn:jn + self.n[i]]))
        return out

    def tape(self, K):
        """Per LP, a (K, 2n + m) numpy array of recorded start iterates."""
        import numpy as np
        sn, sm = int(self.n.sum()), int(self.m.sum())
        per = [[] for _ in range(self.count)]
        for k in range(K):
            x = torch.empty(sn, dtype=torch.float64, device=self.device)
            y = torch.empty(sm, dtype=torch.float64, device=self.device)
            s = torch.empty(sn, dtype=torch.float64, device=self.device)
            capi.check(capi.lp_batch_tape_row(self.h, k, _p(x), _p(y), _p(s)), "lp_batch_tape_row")
            x, y, s = x.cpu().numpy(), y.cpu().numpy(), s.cpu().numpy()
            for i in range(self.count):
                jn, jm = self.v_off_n[i], self.v_off_m[i]
                per[i].append(np.concatenate([x[jn:jn + self.n[i]], y[jm:jm + self.m[i]],
                                              s[jn:jn + self.n[i]]]))
        return [np.stack(r) for r in per]

    def backward(self, xbar, ybar=None, sbar=None):
        """Packed gradients (dict A, b, c, x0, y0, s0) of a loss on the final
        iterates; xbar (and ybar, sbar) packed like iterates()."""
        dev = self.device
        f = lambda k: torch.empty(k, dtype=torch.float64, device=dev)
        sn, sm = int(self.n.sum()), int(self.m.sum())
        out = dict(A=torch.zeros_like(self.A), b=f(sm), c=f(sn), x0=f(sn), y0=f(sm), s0=f(sn))
        xbar = xbar.contiguous().to(torch.float64)
        ybar = None if ybar is None else ybar.contiguous().to(torch.float64)
        sbar = None if sbar is None else sbar.contiguous().to(torch.float64)
        st = capi.lp_batch_backward(self.h, _p(xbar), _p(ybar), _p(sbar), _p(out["A"]),
                                    _p(out["b"]), _p(out["c"]), _p(out["x0"]), _p(out["y0"]),
                                    _p(out["s0"]))
        capi.check(st, "lp_batch_backward")
        return out

    def close(self):
        if getattr(self, "h", None):
            capi.lp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _lp_backward(lp, xbar, ybar=None, sbar=None):
    """Gradients of a loss on the final iterate with respect to the setup
    inputs (lp_backward).  Returns dict A, b, c, x0, y0, s0 of tensors."""
    m, n, dev = lp.m, lp.n, lp.device
    out = dict(A=torch.empty((m, n), dtype=torch.float64, device=dev),
               b=torch.empty(m, dtype=torch.float64, device=dev),
               c=torch.empty(n, dtype=torch.float64, device=dev),
               x0=torch.empty(n, dtype=torch.float64, device=dev),
               y0=torch.empty(m, dtype=torch.float64, device=dev),
               s0=torch.empty(n, dtype=torch.float64, device=dev))
    xbar = xbar.contiguous().to(torch.float64)
    ybar = None if ybar is None else ybar.contiguous().to(torch.float64)
    sbar = None if sbar is None else sbar.contiguous().to(torch.float64)
    st = capi.lp_backward(lp.h, _p(xbar), _p(ybar), _p(sbar), _p(out["A"]), _p(out["b"]),
                          _p(out["c"]), _p(out["x0"]), _p(out["y0"]), _p(out["s0"]))
    capi.check(st, "lp_backward")
    return out


LP.backward = _lp_backward


class PDASFixedK(torch.autograd.Function):
    """x_K after exactly K Section 3 steps from (x0, y0, s0), differentiable with
    respect to A, b, c, x0, y0, s0 (the reverse sweep recomputes every step and
    reuses its Cholesky factor).  The forward stops early only at a psi == 1
    step or an error, which raise."""

    @staticmethod
    def forward(ctx, A, b, c, x0, y0, s0, K, alpha=0.9):
        lp = LP(A.detach().contiguous(), b.detach().contiguous(), c.detach().contiguous(),
                x0.detach().contiguous(), y0.detach().contiguous(), s0.detach().contiguous(),
                alpha=alpha, tape_capacity=int(K))
        res = lp.solve(0.0, int(K))
        if res["status"] != capi.LP_MAX_ITER or res["iters"] != int(K):
            raise RuntimeError(f"fixed-K run stopped early: {capi.status_string(res['status'])}")
        x, y, s = lp.iterate_values()
        ctx.lp = lp
        ctx.keep = (A, b, c, x0, y0, s0)
        return x

    @staticmethod
    def backward(ctx, gx):
        g = ctx.lp.backward(gx)
        ctx.lp.close()
        return g["A"], g["b"], g["c"], g["x0"], g["y0"], g["s0"], None, None
