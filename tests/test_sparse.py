"""Sparse A (canonical CSR, lp_setup_csr / lp_normal_matrix_csr) against the
CPU oracle run on the densified matrix.

The sparse path differs from the dense one only in how the products A w,
A^T v and A D A^T are summed (over the stored entries, in a fixed order),
so the bars are those of the dense path:
  * normal matrix entries: |M_gpu - M_orc| <= 4 n u (|A| D |A|^T)_ij (each
    entry is a dot product of at most n terms);
  * dy on the same input iterate: ||dy_gpu - dy_orc|| / ||dy_orc|| <=
    max(1e-10, 10 m u kappa(M));
  * whole solve: same status and K, b^T y within 1e-9 relative.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1502_03543_amd import capi, lpgen

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu tests need a ROCm GPU")
    capi.load()
    return torch, torch.device("cuda:0")


def _t(torch, dev, a, dtype=None):
    import torch as _torch
    dt = dtype or _torch.float64
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)


def _csr(torch, dev, lp):
    return (_t(torch, dev, lp.row_ptr, torch.int64), _t(torch, dev, lp.col_idx, torch.int32),
            _t(torch, dev, lp.vals))


def _vecs(torch, dev, lp):
    return [_t(torch, dev, v) for v in (lp.b, lp.c, lp.x0, lp.y0, lp.s0)]


def _sparse_lp(torch, dev, lp, **opts):
    from paper_1502_03543_amd import solver
    return solver.CsrLP(*_csr(torch, dev, lp), (lp.m, lp.n), *_vecs(torch, dev, lp), **opts)


@pytest.mark.parametrize("m,n,density,seed", [(64, 256, 0.05, 0), (300, 1200, 0.02, 1),
                                              (517, 1100, 0.01, 2), (130, 517, 0.6, 3)])
def test_csr_normal_matrix(torch_dev, m, n, density, seed):
    """Every lower entry against the oracle's dense product; upper untouched."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_sparse_lp(m, n, density, seed)
    d = np.random.default_rng(seed + 50).uniform(1e-3, 1e3, n)
    print(f"csr normal matrix m={m} n={n} density={density} nnz={lp.nnz}", flush=True)
    Mg = solver.normal_matrix_csr(*_csr(torch, dev, lp), (m, n), _t(torch, dev, d)).cpu().numpy()
    Mo = oracle.normal_matrix(lp.A, d)
    bound = 4 * n * U * (np.abs(lp.A) @ (d[:, None] * np.abs(lp.A.T)))
    low = np.tril(np.ones((m, m), dtype=bool))
    err = np.abs(Mg - Mo)
    assert np.all(err[low] <= bound[low]), float(np.max(err[low] / np.maximum(bound[low], 1e-300)))
    assert np.all(Mg[~low] == 0.0)


@pytest.mark.parametrize("m,n,density,seed", [(64, 256, 0.05, 0), (300, 1200, 0.02, 1),
                                              (700, 2800, 0.01, 4)])
def test_csr_iteration_parity(torch_dev, m, n, density, seed):
    """Each step on the GPU's own input iterate against oracle.iterate."""
    torch, dev = torch_dev
    lp = lpgen.gen_sparse_lp(m, n, density, seed)
    print(f"csr iteration parity m={m} n={n} density={density}", flush=True)
    h = _sparse_lp(torch, dev, lp, alpha=0.95)
    steps = 0
    for k in range(100):
        x, y, s = (v.cpu().numpy() for v in h.iterate_values())
        if x @ s < 1e-8:
            break
        info = h.iterate()
        _, dyg, _ = (v.cpu().numpy() for v in h.direction())
        it = oracle.iterate(lp.A, lp.b, lp.c, x, y, s, 0.95)
        assert info["status"] == capi.LP_OK and it.status == oracle.CONTINUE, (k, info, it.status)
        kap = np.linalg.cond(it.M)
        tol = max(1e-10, 10 * m * U * kap)
        rel = np.linalg.norm(dyg - it.dy) / np.linalg.norm(it.dy)
        assert rel <= tol, (k, rel, tol, kap)
        assert abs(info["psi"] - it.psi) <= tol * it.psi, (k, info["psi"], it.psi)
        if abs(info["psi"] - it.psi) <= 1e-14 * it.psi:
            assert info["argmax"] == it.argmax
        xn, yn, sn = (v.cpu().numpy() for v in h.iterate_values())
        assert np.all(xn > 0) and np.all(sn > 0)
        np.testing.assert_allclose(xn, it.x, rtol=0, atol=tol * np.max(np.abs(it.x)) * 10)
        np.testing.assert_allclose(yn, it.y, rtol=0, atol=tol * np.max(np.abs(it.y)) * 10 + 1e-12)
        steps += 1
    assert steps >= 10


@pytest.mark.parametrize("m,n,density,seed", [(1, 2, 1.0, 0), (64, 256, 0.05, 5),
                                              (257, 1100, 0.02, 6), (1000, 4000, 0.005, 7)])
def test_csr_solve_parity(torch_dev, m, n, density, seed):
    """Whole loop: status, K and b^T y as the oracle on the dense form."""
    torch, dev = torch_dev
    lp = lpgen.gen_sparse_lp(m, n, density, seed)
    print(f"csr solve parity m={m} n={n} density={density} nnz={lp.nnz}", flush=True)
    h = _sparse_lp(torch, dev, lp, alpha=0.95)
    res = h.solve(1e-8, 200)
    ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
    assert capi.status_string(res["status"]) == "LP_" + ro.status_name
    if ro.status == oracle.CONVERGED:
        assert res["iters"] == ro.iters
        x, y, s = (v.cpu().numpy() for v in h.iterate_values())
        assert abs(lp.b @ y - lp.b @ ro.y) <= 1e-9 * max(1.0, abs(lp.b @ ro.y))
        assert x @ s < 1e-8 and np.all(x > 0) and np.all(s > 0)


def test_csr_matches_dense_path(torch_dev):
    """The same LP through lp_setup and lp_setup_csr: same status and K,
    the first ten psi within 1e-9 (later iterates drift apart by rounding
    that the ill-conditioned late systems amplify; each step's own parity is
    checked against the oracle above) and the objective within 1e-9."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_sparse_lp(400, 1600, 0.02, 8)
    hs = _sparse_lp(torch, dev, lp, alpha=0.95)
    hd = solver.LP(*[_t(torch, dev, v) for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)],
                   alpha=0.95)
    rs = hs.solve(1e-8, 200, want_log=True)
    rd = hd.solve(1e-8, 200, want_log=True)
    assert rs["status"] == rd["status"] == capi.LP_CONVERGED
    assert rs["iters"] == rd["iters"]
    for a, b in list(zip(rs["log"], rd["log"]))[:10]:
        assert abs(a["psi"] - b["psi"]) <= 1e-9 * b["psi"], (a["psi"], b["psi"])
    assert abs(rs["dual_obj"] - rd["dual_obj"]) <= 1e-9 * max(1.0, abs(rd["dual_obj"]))


def test_csr_predictor_corrector(torch_dev):
    """LP_METHOD_PC on a CSR matrix against the oracle's predictor-corrector."""
    torch, dev = torch_dev
    lp = lpgen.gen_sparse_lp(200, 800, 0.03, 9)
    h = _sparse_lp(torch, dev, lp, alpha=0.95, method="pc")
    res = h.solve(1e-8, 100)
    ro = oracle.pc_solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 100)
    assert capi.status_string(res["status"]) == "LP_" + ro.status_name == "LP_CONVERGED"
    assert res["iters"] == ro.iters
    _, y, _ = (v.cpu().numpy() for v in h.iterate_values())
    assert abs(lp.b @ y - lp.b @ ro.y) <= 1e-9 * max(1.0, abs(lp.b @ ro.y))


def test_csr_determinism(torch_dev):
    torch, dev = torch_dev
    lp = lpgen.gen_sparse_lp(300, 1200, 0.02, 10)
    outs = []
    for _ in range(2):
        h = _sparse_lp(torch, dev, lp, alpha=0.95)
        h.solve(1e-8, 10)
        outs.append([v.cpu().numpy() for v in h.iterate_values()])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_csr_errors(torch_dev):
    """Bad CSR structure or values, an empty matrix, options the sparse path
    does not take, and the backward call without a tape."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_sparse_lp(64, 256, 0.05, 11)
    rp, ci, v = lp.row_ptr.copy(), lp.col_idx.copy(), lp.vals.copy()
    r = int(np.argmax(np.diff(rp)))
    ci_unsorted = ci.copy()
    ci_unsorted[rp[r]], ci_unsorted[rp[r] + 1] = ci[rp[r] + 1], ci[rp[r]]
    ci_range = ci.copy()
    ci_range[-1] = lp.n
    v_nan = v.copy()
    v_nan[3] = np.nan
    rp_bad = rp.copy()
    rp_bad[r + 1] = rp[r] - 1
    for name, (a, b, c) in {"unsorted": (rp, ci_unsorted, v), "range": (rp, ci_range, v),
                            "nan": (rp, ci, v_nan), "row_ptr": (rp_bad, ci, v)}.items():
        print(f"csr error case {name}", flush=True)
        T = (_t(torch, dev, a, torch.int64), _t(torch, dev, b, torch.int32), _t(torch, dev, c))
        with pytest.raises(RuntimeError, match="LP_ERR_INVALID_ARG"):
            solver.CsrLP(*T, (lp.m, lp.n), *_vecs(torch, dev, lp))
    # an empty A: setup succeeds, the first normal matrix is zero
    T = (torch.zeros(lp.m + 1, dtype=torch.int64, device=dev),
         torch.zeros(0, dtype=torch.int32, device=dev),
         torch.zeros(0, dtype=torch.float64, device=dev))
    h = solver.CsrLP(*T, (lp.m, lp.n), *_vecs(torch, dev, lp))
    assert h.iterate()["status"] == capi.LP_ERR_BREAKDOWN
    h = _sparse_lp(torch, dev, lp)
    xb = torch.ones(lp.n, dtype=torch.float64, device=dev)
    st = capi.lp_backward(h.h, xb.data_ptr(), None, None, None, None, None, None, None, None)
    assert st == capi.LP_ERR_NO_TAPE
    x0 = _vecs(torch, dev, lp)
    x0[2][5] = -1.0
    with pytest.raises(RuntimeError, match="LP_ERR_NOT_INTERIOR"):
        solver.CsrLP(*_csr(torch, dev, lp), (lp.m, lp.n), *x0)


def _golden(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    if name.endswith(".npy"):
        return np.load(path)
    with open(path) as f:
        return json.load(f)


def test_csr_full_size_lp2048x8192(torch_dev):
    """The sparse benchmark instance (m=2048, n=8192, density 1%, seed 0):
    sampled normal-matrix entries against exact dot products, the first
    direction and the whole solve against the oracle's record."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    m, n = 2048, 8192
    gold = _golden("lp2048x8192_d01_seed0_csr.json")
    dy0 = _golden("lp2048x8192_d01_seed0_csr_dy0.npy")
    lp = lpgen.gen_sparse_lp(m, n, 0.01, 0)
    assert lp.nnz == gold["nnz"]
    d = lp.x0 / lp.s0
    print("csr full size: normal matrix samples", flush=True)
    Mg = solver.normal_matrix_csr(*_csr(torch, dev, lp), (m, n), _t(torch, dev, d)).cpu().numpy()
    rng = np.random.default_rng(1)
    ii = rng.integers(0, m, 3000)
    jj = rng.integers(0, m, 3000)
    ii, jj = np.maximum(ii, jj), np.minimum(ii, jj)
    ii = np.concatenate([ii, [m - 1, m - 1, 0, 2047]])
    jj = np.concatenate([jj, [0, m - 1, 0, 1920]])
    for i, j in zip(ii, jj):
        ref = float(np.dot(lp.A[i] * d, lp.A[j]))
        bound = 4 * n * U * float(np.dot(np.abs(lp.A[i]) * d, np.abs(lp.A[j])))
        assert abs(Mg[i, j] - ref) <= bound, (i, j, Mg[i, j], ref)
    print("csr full size: first direction and whole solve", flush=True)
    h = _sparse_lp(torch, dev, lp, alpha=0.95)
    info = h.iterate()
    assert info["status"] == capi.LP_OK
    _, dyg, _ = (v.cpu().numpy() for v in h.direction())
    rel = np.linalg.norm(dyg - dy0) / np.linalg.norm(dy0)
    print(f"first dy relative difference {rel:.2e}", flush=True)
    assert rel <= 1e-10, rel
    res = h.solve(1e-8, 200)
    K = res["iters"] + 1
    print(f"GPU: {capi.status_string(res['status'])} K={K} b^T y={res['dual_obj']!r}; oracle: "
          f"{gold['status']} K={gold['iters']} b^T y={gold['dual_obj']!r}", flush=True)
    assert capi.status_string(res["status"]) == "LP_" + gold["status"] == "LP_CONVERGED"
    assert K == gold["iters"]
    assert abs(res["dual_obj"] - gold["dual_obj"]) <= 1e-9 * max(1.0, abs(gold["dual_obj"]))
    x, y, s = (v.cpu().numpy() for v in h.iterate_values())
    assert x @ s < 1e-8 and np.all(x > 0) and np.all(s > 0)
    assert np.linalg.norm(lp.A @ x - lp.b) <= 1e-8 * np.linalg.norm(lp.b)


def test_csr_max_rows_normal_matrix(torch_dev):
    """m = LP_CSR_MAX_M (the LDS row at its largest): sampled entries of
    A D A^T against the oracle's product of the two rows involved."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    m, n, per_row = 16384, 20000, 12
    rng = np.random.default_rng(12)
    cols = np.sort(np.stack([rng.choice(n, per_row, replace=False) for _ in range(m)]), axis=1)
    rp = np.arange(0, m * per_row + 1, per_row, dtype=np.int64)
    ci = cols.reshape(-1).astype(np.int32)
    v = rng.standard_normal(m * per_row)
    d = rng.uniform(0.1, 10.0, n)
    print("csr normal matrix m=16384", flush=True)
    Mg = solver.normal_matrix_csr(_t(torch, dev, rp, torch.int64), _t(torch, dev, ci, torch.int32),
                                  _t(torch, dev, v), (m, n), _t(torch, dev, d))
    ii = np.concatenate([rng.integers(0, m, 400), [m - 1, m - 1, 0]])
    jj = np.concatenate([rng.integers(0, m, 400), [0, m - 1, 0]])
    ii, jj = np.maximum(ii, jj), np.minimum(ii, jj)
    got = Mg[torch.from_numpy(ii).to(dev), torch.from_numpy(jj).to(dev)].cpu().numpy()
    for t, (i, j) in enumerate(zip(ii, jj)):
        R = np.zeros((2, n))
        R[0, cols[i]] = v[i * per_row:(i + 1) * per_row]
        R[1, cols[j]] = v[j * per_row:(j + 1) * per_row]
        ref = oracle.normal_matrix(R, d)[1, 0] if i != j else oracle.normal_matrix(R[:1], d)[0, 0]
        bound = 4 * per_row * U * float(np.abs(R[0]) @ (d * np.abs(R[1]))) + 1e-300
        assert abs(got[t] - ref) <= bound, (i, j, got[t], ref)
    assert float(Mg.triu(1).abs().max()) == 0.0
