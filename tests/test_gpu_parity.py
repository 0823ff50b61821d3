"""GPU path (libpdas through its C ABI) against the CPU oracle.

Tolerances (derived from the arithmetic; see the design notes):
  * normal matrix entries: each is a length-n dot product, so
    |M_gpu - M_orc| <= 4 n u (|A| D |A|^T)_ij;
  * dy on the same input iterate: ||dy_gpu - dy_orc|| / ||dy_orc|| <=
    max(1e-10, 10 m u kappa(M)) (the strict 1e-10 wherever kappa u <= 1e-12);
  * final dual objective b^T y within 1e-9 max(1, |b^T y|), same status and K.
"""
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


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


def _lp_tensors(torch, dev, lp):
    return [_t(torch, dev, v) for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]


SHAPES = [(64, 256), (100, 333), (130, 517), (257, 1100), (700, 1500)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_normal_matrix(torch_dev, m, n):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    rng = np.random.default_rng(m * 7 + n)
    A = rng.standard_normal((m, n))
    d = rng.uniform(1e-3, 1e3, n)
    print(f"normal_matrix m={m} n={n}", flush=True)
    Mg = solver.normal_matrix(_t(torch, dev, A), _t(torch, dev, d)).cpu().numpy()
    Mo = oracle.normal_matrix(A, d)
    bound = 4 * n * U * (np.abs(A) @ (d[:, None] * np.abs(A.T)))
    low = np.tril(np.ones((m, m), dtype=bool))
    err = np.abs(Mg - Mo)
    assert np.all(err[low] <= bound[low]), float(np.max(err[low] / bound[low]))
    assert np.all(Mg[~low] == 0.0)  # upper triangle untouched


@pytest.mark.parametrize("m", [1, 64, 100, 200, 333, 700, 4096, 4133])
def test_cholesky_and_solve(torch_dev, m):
    """Factor and solve against the oracle; m = 4096 (the threshold, whole
    groups) and 4133 (ending in a ragged group) take the grouped schedule of
    large matrices (panels by four, each group's update of the columns
    beyond the next group on a second stream) and are factored twice to the
    same bits."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    rng = np.random.default_rng(m)
    B = rng.standard_normal((m, 2 * m + 3))
    M = B @ B.T + m * np.eye(m)
    print(f"cholesky m={m}", flush=True)
    Lg, fail, minp, st = solver.cholesky(_t(torch, dev, np.tril(M)))
    assert st == capi.LP_OK and fail == -1
    Lg = Lg.cpu().numpy()
    if m >= 4096:
        # the grouped schedule's two streams: the factor is the same bit for
        # bit from one run to the next
        Lg2, _, _, _ = solver.cholesky(_t(torch, dev, np.tril(M)))
        assert np.array_equal(Lg, Lg2.cpu().numpy())
    Lo, fo, mpo = oracle.cholesky(M)
    assert fo == -1
    kappa = np.linalg.cond(M)
    assert np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo) <= max(1e-13, 10 * m * U * kappa)
    # element by element, against the scale of the entry's row (||L_i,:|| =
    # sqrt(M_ii)): both factors are backward stable, so they differ by the
    # conditioning times the unit roundoff
    row = np.sqrt(np.diag(M))[:, None]
    elt = np.abs(Lg - Lo) / row
    assert np.all(elt <= max(1e-14, 10 * m * U * kappa)), float(elt.max())
    assert np.all(np.triu(Lg, 1) == 0.0)
    assert np.linalg.norm(Lg @ Lg.T - M) / np.linalg.norm(M) <= 10 * m * U
    assert abs(minp - mpo) <= 1e-12 * mpo
    r = rng.standard_normal(m)
    wg = solver.chol_solve(_t(torch, dev, Lg), _t(torch, dev, r)).cpu().numpy()
    wo = oracle.cholesky_solve(Lo, r)
    assert np.linalg.norm(wg - wo) / np.linalg.norm(wo) <= max(1e-12, 10 * m * U * kappa)


def test_cholesky_breakdown_indefinite(torch_dev):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    m = 150
    rng = np.random.default_rng(5)
    B = rng.standard_normal((m, 2 * m))
    M = B @ B.T
    M[77, 77] = -1.0
    _, fail, _, st = solver.cholesky(_t(torch, dev, np.tril(M)))
    _, fo, _ = oracle.cholesky(M)
    assert st == capi.LP_ERR_BREAKDOWN and fail == fo == 77


def _kappa(Mo):
    return np.linalg.cond(Mo)


@pytest.mark.parametrize("m,n,seed", [(64, 256, 0), (100, 333, 1), (130, 517, 2),
                                      (700, 2800, 3)])
def test_iteration_parity(torch_dev, m, n, seed):
    """Every step on the GPU's own input iterate: dy, psi, argmax, t and the
    new iterate against oracle.iterate on the same bytes."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(m, n, seed)
    print(f"iteration parity m={m} n={n} seed={seed}", flush=True)
    h = solver.LP(*_lp_tensors(torch, dev, lp), alpha=0.95)
    strict = 0
    for k in range(100):
        x, y, s = (v.cpu().numpy() for v in h.iterate_values())
        if x @ s < 1e-8:
            break
        info = h.iterate()
        dxg, dyg, dsg = (v.cpu().numpy() for v in h.direction())
        it = oracle.iterate(lp.A, lp.b, lp.c, x, y, s, 0.95)
        assert info["status"] == capi.LP_OK and it.status == oracle.CONTINUE, (k, info, it.status)
        kap = _kappa(it.M)
        tol = max(1e-10, 10 * m * U * kap)
        if kap * U <= 1e-12:
            strict += 1
        rel = np.linalg.norm(dyg - it.dy) / np.linalg.norm(it.dy)
        assert rel <= tol, (k, rel, tol, kap)
        # residual of the GPU direction in the oracle's system, against the
        # componentwise bound of forming M and rhs (length-n dot products) and
        # of a backward-stable Cholesky solve (size m)
        absA = np.abs(lp.A)
        res = np.linalg.norm(it.rhs - it.M @ dyg)
        bound = 10 * U * (n * np.linalg.norm(absA @ (it.d * (absA.T @ np.abs(dyg))))
                          + m * np.linalg.norm(it.M, 2) * np.linalg.norm(dyg)
                          + n * np.linalg.norm(np.abs(lp.b) + absA @ (it.d * (
                              np.abs(lp.c) + absA.T @ np.abs(y) + s))))
        assert res <= bound, (k, res, bound)
        assert abs(info["psi"] - it.psi) <= tol * it.psi, (k, info["psi"], it.psi)
        if abs(info["psi"] - it.psi) <= 1e-14 * it.psi:
            assert info["argmax"] == it.argmax
        xn, yn, sn = (v.cpu().numpy() for v in h.iterate_values())
        assert np.all(xn > 0) and np.all(sn > 0)
        np.testing.assert_allclose(xn, it.x, rtol=0, atol=tol * np.max(np.abs(it.x)) * 10)
        np.testing.assert_allclose(yn, it.y, rtol=0, atol=tol * np.max(np.abs(it.y)) * 10 + 1e-12)
        np.testing.assert_allclose(info["gap_after"], it.x @ it.s, rtol=max(1e-9, 100 * tol))
    assert strict >= 3


@pytest.mark.parametrize("m,n,seed", [(64, 256, 0), (64, 256, 1), (64, 256, 2), (100, 333, 3),
                                      (130, 517, 4), (257, 1100, 5), (1024, 4096, 6)])
def test_solve_parity(torch_dev, m, n, seed):
    """Whole Section 3 loop to x^T s < 1e-8: same status and iteration count
    as the oracle, dual objective within 1e-9 relative."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(m, n, seed)
    print(f"solve parity m={m} n={n} seed={seed}", flush=True)
    h = solver.LP(*_lp_tensors(torch, dev, lp), alpha=0.95)
    res = h.solve(1e-8, 200)
    ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
    assert capi.status_string(res["status"]) == "LP_" + ro.status_name
    x, y, s = (v.cpu().numpy() for v in h.iterate_values())
    if ro.status == oracle.CONVERGED:
        assert res["iters"] == ro.iters
        by, byo = lp.b @ y, lp.b @ ro.y
        assert abs(by - byo) <= 1e-9 * max(1.0, abs(byo)), (by, byo)
        assert abs(res["dual_obj"] - by) <= 1e-12 * max(1.0, abs(by))
        cx, cxo = lp.c @ x, lp.c @ ro.x
        rp = np.linalg.norm(lp.A @ x - lp.b)
        assert abs(cx - cxo) <= 1e-9 * max(1.0, abs(cxo)) + 2 * np.linalg.norm(y) * rp
        assert x @ s < 1e-8 and np.all(x > 0) and np.all(s > 0)
        assert abs(res["gap"] - x @ s) <= 1e-12 + 1e-9 * (x @ s)


def test_psi1_worked_example(torch_dev):
    """Section 3, psi == 1 branch; exact in binary floating point."""
    import json
    import os
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "psi1_example.json")))
    e = g["expect"]
    T = [_t(torch, dev, np.array(g[k], dtype=np.float64)) for k in ("A", "b", "c", "x0", "y0", "s0")]
    h = solver.LP(*T, alpha=g["alpha"])
    info = h.iterate()
    assert capi.status_string(info["status"]) == "LP_" + e["status"]
    assert info["psi"] == e["psi"] and info["argmax"] == e["argmax"] and info["t"] == e["t"]
    dx, dy, ds = (v.cpu().numpy() for v in h.direction())
    assert list(dx) == e["dx"] and list(dy) == e["dy"] and list(ds) == e["ds"]
    x, y, s = (v.cpu().numpy() for v in h.iterate_values())
    assert list(x) == e["x1"] and list(y) == e["y1"] and list(s) == e["s1"]


@pytest.mark.parametrize("case", ["shape", "not_interior", "nan", "alpha", "max_iter",
                                  "zero_row_breakdown"])
def test_status_cases(torch_dev, case):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(16, 48, 0)
    A, b, c, x0, y0, s0 = lp.A.copy(), lp.b.copy(), lp.c.copy(), lp.x0.copy(), lp.y0.copy(), lp.s0.copy()
    alpha, max_iter = 0.95, 100
    if case == "shape":
        A, c, x0, s0 = np.ascontiguousarray(A[:, :16]), c[:16], x0[:16], s0[:16]
    elif case == "not_interior":
        s0[7] = 0.0
    elif case == "nan":
        b[3] = np.nan
    elif case == "alpha":
        alpha = 1.0
    elif case == "max_iter":
        max_iter = 2
    elif case == "zero_row_breakdown":
        A[5] = 0.0
        b = A @ x0
    ro = oracle.solve(A, b, c, x0, y0, s0, alpha, 1e-8, max_iter)
    T = [_t(torch, dev, v) for v in (A, b, c, x0, y0, s0)]
    try:
        h = solver.LP(*T, alpha=alpha)
    except RuntimeError as err:
        assert str(err).endswith("LP_" + ro.status_name), (str(err), ro.status_name)
        return
    res = h.solve(1e-8, max_iter)
    assert capi.status_string(res["status"]) == "LP_" + ro.status_name
    assert res["iters"] == ro.iters
    if case == "zero_row_breakdown":
        x, y, s = (v.cpu().numpy() for v in h.iterate_values())
        np.testing.assert_array_equal(x, x0)  # last valid iterate kept


def test_determinism(torch_dev):
    """Fixed-order reductions: two runs give bitwise identical iterates."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(300, 1000, 7)
    outs = []
    for _ in range(2):
        h = solver.LP(*_lp_tensors(torch, dev, lp), alpha=0.95)
        h.solve(1e-8, 8)
        outs.append([v.cpu().numpy() for v in h.iterate_values()])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_profiling_levels(torch_dev):
    """Timing events change no result: an unprofiled solve, one timing only
    the normal-matrix kernel (two events per iteration) and one timing every
    phase give bitwise identical iterates; the kernel-only level reports that
    kernel's time for every iteration and no phase times."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(600, 1500, 11)
    outs, tims = [], []
    for prof in (False, "kernel", True):
        h = solver.LP(*_lp_tensors(torch, dev, lp), alpha=0.95, profile=prof)
        r = h.solve(1e-8, 6)
        outs.append([v.cpu().numpy() for v in h.iterate_values()])
        tims.append((r["iters"], h.timings()))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            np.testing.assert_array_equal(a, b)
    k, tk = tims[1]
    assert tk["iterations"] == k == tk["normal_launches"] and k > 0
    assert tk["normal_kernel_ms"] > 0
    assert tk["potrf_ms"] == tk["trsv_ms"] == tk["iter_ms"] == tk["normal_ms"] == 0
    _, tf = tims[2]
    assert tf["iter_ms"] > tf["normal_kernel_ms"] > 0 and tf["potrf_ms"] > 0
    assert tims[0][1]["iterations"] == 0


def _golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    if name.endswith(".npy"):
        return np.load(path)
    with open(path) as f:
        return json.load(f)


def test_full_size_lp2048x8192(torch_dev):
    """The benchmark instance (m=2048, n=8192, seed 0) in the benchmark's
    launch configuration: sampled normal-matrix entries against exact dot
    products; the first direction and the whole solve (status, K, b^T y)
    against the oracle's, stored by tests/golden/make_golden.py; and
    properties that hold at any size."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    m, n = 2048, 8192
    gold = _golden("lp2048x8192_seed0.json")
    dy0 = _golden("lp2048x8192_seed0_dy0.npy")
    lp = lpgen.gen_lp(m, n, 0)
    T = _lp_tensors(torch, dev, lp)
    print("full size: normal matrix samples", flush=True)
    d = lp.x0 / lp.s0
    Mg = solver.normal_matrix(T[0], _t(torch, dev, d)).cpu().numpy()
    rng = np.random.default_rng(0)
    ii = rng.integers(0, m, 3000)
    jj = rng.integers(0, m, 3000)
    ii, jj = np.maximum(ii, jj), np.minimum(ii, jj)
    ii = np.concatenate([ii, [m - 1, m - 1, 0, 1919, 2047]])
    jj = np.concatenate([jj, [0, m - 1, 0, 1792, 1920]])
    for i, j in zip(ii, jj):
        ref = float(np.dot(lp.A[i] * d, lp.A[j]))
        bound = 4 * n * U * float(np.dot(np.abs(lp.A[i]) * d, np.abs(lp.A[j])))
        assert abs(Mg[i, j] - ref) <= bound, (i, j, Mg[i, j], ref)
    print("full size: first direction vs oracle", flush=True)
    h = solver.LP(*T, alpha=0.95)
    info = h.iterate()
    assert info["status"] == capi.LP_OK
    _, dyg, _ = (v.cpu().numpy() for v in h.direction())
    fd = gold["first_direction"]
    rel = np.linalg.norm(dyg - dy0) / np.linalg.norm(dy0)
    print(f"first dy relative difference {rel:.2e}", flush=True)
    assert rel <= 1e-10, rel
    assert abs(info["psi"] - fd["psi"]) <= 1e-10 * fd["psi"] and info["argmax"] == fd["argmax"]
    print("full size: whole solve", flush=True)
    res = h.solve(1e-8, 200, want_log=True)
    K = res["iters"] + 1
    by = res["dual_obj"]
    print(f"GPU: {capi.status_string(res['status'])} K={K} b^T y={by!r}; oracle: "
          f"{gold['status']} K={gold['iters']} b^T y={gold['dual_obj']!r}", flush=True)
    psi_g = [info["psi"]] + [e["psi"] for e in res["log"]]
    psi_o = [e["psi"] for e in gold["log"]]
    dpsi = [abs(a - b) / b for a, b in zip(psi_g, psi_o)]
    print("psi relative difference per iteration:", ["%.0e" % v for v in dpsi], flush=True)
    assert capi.status_string(res["status"]) == "LP_" + gold["status"] == "LP_CONVERGED"
    assert K == gold["iters"], (K, gold["iters"])
    assert abs(by - gold["dual_obj"]) <= 1e-9 * max(1.0, abs(gold["dual_obj"]))
    x, y, s = (v.cpu().numpy() for v in h.iterate_values())
    gap = x @ s
    assert gap < 1e-8 and np.all(x > 0) and np.all(s > 0)
    assert abs(lp.b @ y - by) <= 1e-12 * max(1.0, abs(by))
    assert np.linalg.norm(lp.A @ x - lp.b) <= 1e-8 * np.linalg.norm(lp.b)
    assert np.linalg.norm(lp.A.T @ y + s - lp.c) <= 1e-11 * np.linalg.norm(lp.c)
    # c^T x - b^T y = x^T s + y^T r_p + x^T r_d: the identity holds up to the
    # residuals that remain (the primal residual floor of a late iterate)
    rp, rd = lp.A @ x - lp.b, lp.c - lp.A.T @ y - s
    slack = np.abs(y) @ np.abs(rp) + np.abs(x) @ np.abs(rd)
    assert abs((lp.c @ x - lp.b @ y) - gap) <= slack + 1e-9 * max(1.0, abs(lp.c @ x))
    for e in res["log"]:
        # psi >= 1 and gap+ = (1 - alpha/psi) gap on (nearly) feasible iterates
        assert e["psi"] >= 1 - 1e-6 and e["gap_after"] < e["gap_before"]
        if e["gap_before"] > 1e-4:
            assert abs(e["gap_after"] - (1 - 0.95 / e["psi"]) * e["gap_before"]) <= 1e-3 * e["gap_after"]
