"""lp_chol_solve_noalloc (scratch in a fixed device array, no workspace)
against lp_chol_solve (caller's workspace) through the C ABI: two calls in a
row, the second smaller, each bit-identical to the workspace form and within
the solve's error bound of the CPU oracle."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1502_03543_amd import capi

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _spd(m, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((m, 2 * m + 5))
    return B @ B.T + m * np.eye(m), rng.standard_normal(m)


def test_noalloc_chol_solve_matches_workspace_form():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a ROCm GPU")
    lib = capi.load()
    fn = lib.lp_chol_solve_noalloc
    fn.restype = C.c_int32
    fn.argtypes = [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    dev = torch.device("cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for m, seed in ((1100, 0), (333, 1)):  # second call smaller: stale scratch must not leak
        print(f"noalloc solve m={m}", flush=True)
        M, r = _spd(m, seed)
        Lo, fail, _ = oracle.cholesky(M)
        assert fail == -1
        L = torch.from_numpy(np.ascontiguousarray(Lo)).to(dev)
        rt = torch.from_numpy(r).to(dev)
        y_na = torch.full((m,), np.nan, dtype=torch.float64, device=dev)
        y_ws = torch.full((m,), np.nan, dtype=torch.float64, device=dev)
        size = C.c_size_t(0)
        assert capi.lp_blocks_workspace_size(m, m + 1, C.byref(size)) == capi.LP_OK
        ws = torch.empty(size.value + 256, dtype=torch.uint8, device=dev)
        addr = (ws.data_ptr() + 255) // 256 * 256
        st = fn(m, L.data_ptr(), m, rt.data_ptr(), y_na.data_ptr(), stream)
        assert st == capi.LP_OK, capi.status_string(st)
        st = capi.lp_chol_solve(m, C.c_void_p(L.data_ptr()), m, C.c_void_p(rt.data_ptr()),
                                C.c_void_p(y_ws.data_ptr()), C.c_void_p(addr), size.value,
                                stream)
        assert st == capi.LP_OK
        torch.cuda.synchronize()
        a, b = y_na.cpu().numpy(), y_ws.cpu().numpy()
        np.testing.assert_array_equal(a, b)
        wo = oracle.cholesky_solve(Lo, r)
        kappa = np.linalg.cond(M)
        assert np.linalg.norm(a - wo) / np.linalg.norm(wo) <= max(1e-12, 10 * m * U * kappa)
    # sizes beyond the array are refused before any launch
    st = fn(32768 + 64, L.data_ptr(), 32768 + 64, rt.data_ptr(), y_na.data_ptr(), stream)
    assert capi.status_string(st) == "LP_ERR_WORKSPACE"
