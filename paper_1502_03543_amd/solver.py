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
            refine_tol=1e-12, refine_max=5, profile=False) -> capi.lp_options:
    o = capi.lp_options()
    capi.lp_options_default(C.byref(o))
    o.alpha = float(alpha)
    o.precision = _PREC[precision]
    o.tape_capacity = int(tape_capacity)
    o.mixed_switch_gap = float(mixed_switch_gap)
    o.refine_tol = float(refine_tol)
    o.refine_max = int(refine_max)
    o.profile = int(bool(profile))
    return o


class LP:
    """One LP on the GPU (lp_setup ... lp_destroy)."""

    def __init__(self, A, b, c, x0, y0, s0, **opts):
        m, n = A.shape
        for t, shp, nm in ((A, (m, n), "A"), (b, (m,), "b"), (c, (n,), "c"), (x0, (n,), "x0"),
                           (y0, (m,), "y0"), (s0, (n,), "s0")):
            _need(t, shp, nm)
        self.m, self.n = m, n
        self.device = A.device
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
