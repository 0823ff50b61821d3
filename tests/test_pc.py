"""Predictor-corrector variant (LP_METHOD_PC: Mehrotra's method, cited in
the paper's previous-work section) on the GPU against the oracle's
predictor-corrector (oracle.pc_iterate / oracle.pc_solve), same tolerances
as the Section 3 path: each step on the GPU's own input iterate (dy within
max(1e-10, 10 m u kappa(M)), step lengths and centring parameter), and whole
solves with the same status, K and b^T y within 1e-9 relative."""
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


def _T(torch, dev, lp):
    return [torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(dev)
            for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]


@pytest.mark.parametrize("m,n,seed", [(64, 256, 0), (130, 517, 2), (700, 2800, 3)])
def test_pc_iteration_parity(torch_dev, m, n, seed):
    """Each step on the GPU's own input iterate against the long-double
    oracle on the same bytes.  The predictor is the Section 3 direction (its
    bound is the single-solve 10 m u kappa(M)); the corrector also carries the
    predictor's rounding through dx_aff o ds_aff / s and sigma = (mu_aff/mu)^3,
    which late in the run (s_j near 0 for basic j) can exceed that bound.  So
    the corrector is held to max(1e-10, 10 m u kappa, 10 e64), e64 being the
    FP64 oracle's own distance from the long-double oracle at that step."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(m, n, seed)
    print(f"pc iteration parity m={m} n={n} seed={seed}", flush=True)
    h = solver.LP(*_T(torch, dev, lp), alpha=0.95, method="pc")
    rel_of = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    steps = 0
    for k in range(60):
        x, y, s = (v.cpu().numpy() for v in h.iterate_values())
        if x @ s < 1e-8:
            break
        info = h.iterate()
        it = oracle.pc_iterate(lp.A, lp.b, lp.c, x, y, s, 0.95)
        ix = oracle.pc_iterate(lp.A, lp.b, lp.c, x, y, s, 0.95, precision="f80")
        assert info["status"] == capi.LP_OK and it.status == ix.status == oracle.CONTINUE, \
            (k, info, it.status, ix.status)
        _, dyg, _ = (v.cpu().numpy() for v in h.direction())
        ref = oracle.iterate(lp.A, lp.b, lp.c, x, y, s, 0.95)  # its M: conditioning
        kap = np.linalg.cond(ref.M)
        e64 = rel_of(it.dy, ix.dy)
        tol = max(1e-10, 10 * m * U * kap, 10 * e64)
        rel = rel_of(dyg, ix.dy)
        print(f"k={k} kappa {kap:.1e} sigma {ix.sigma:.1e}: dy GPU {rel:.1e}, FP64 oracle "
              f"{e64:.1e}, bound {tol:.1e}", flush=True)
        assert rel <= tol, (k, rel, tol, kap, e64)
        for key, okey in (("alpha_primal", "alpha_p"), ("alpha_dual", "alpha_d"),
                          ("sigma", "sigma")):
            a, b, b64 = info[key], getattr(ix, okey), getattr(it, okey)
            t = max(100 * m * U * kap, 10 * abs(b64 - b) / max(abs(b), 1e-300))
            assert abs(a - b) <= t * max(abs(b), 1e-300), (k, key, a, b, b64)
        xn, yn, sn = (v.cpu().numpy() for v in h.iterate_values())
        assert np.all(xn > 0) and np.all(sn > 0)
        np.testing.assert_allclose(xn, ix.x, rtol=0, atol=10 * tol * np.max(np.abs(ix.x)))
        np.testing.assert_allclose(yn, ix.y, rtol=0, atol=10 * tol * np.max(np.abs(ix.y)) + 1e-12)
        steps += 1
    assert steps >= 8


@pytest.mark.parametrize("m,n,seed", [(64, 256, 0), (64, 256, 1), (64, 256, 2), (257, 1100, 5),
                                      (1024, 4096, 6)])
def test_pc_solve_parity(torch_dev, m, n, seed):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(m, n, seed)
    print(f"pc solve parity m={m} n={n} seed={seed}", flush=True)
    h = solver.LP(*_T(torch, dev, lp), alpha=0.95, method="pc")
    res = h.solve(1e-8, 100)
    ro = oracle.pc_solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 100)
    print(f"GPU {capi.status_string(res['status'])} K={res['iters']}; oracle "
          f"{ro.status_name} K={ro.iters}", flush=True)
    assert capi.status_string(res["status"]) == "LP_" + ro.status_name == "LP_CONVERGED"
    assert res["iters"] == ro.iters
    x, y, s = (v.cpu().numpy() for v in h.iterate_values())
    byo = lp.b @ ro.y
    assert abs(lp.b @ y - byo) <= 1e-9 * max(1.0, abs(byo)), (lp.b @ y, byo)
    assert x @ s < 1e-8 and np.all(x > 0) and np.all(s > 0)
    assert np.linalg.norm(lp.A @ x - lp.b) <= 1e-8 * np.linalg.norm(lp.b)


def test_pc_full_size_lp2048x8192(torch_dev):
    """The benchmark instance under the predictor-corrector variant against the
    oracle's run (tests/golden/make_golden.py c2pc): status, K, b^T y, and the
    affine-scaling optimum."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    with open(os.path.join(gdir, "lp2048x8192_seed0_pc.json")) as f:
        gold = json.load(f)
    with open(os.path.join(gdir, "lp2048x8192_seed0.json")) as f:
        affine = json.load(f)
    lp = lpgen.gen_lp(2048, 8192, 0)
    h = solver.LP(*_T(torch, dev, lp), alpha=0.95, method="pc")
    res = h.solve(1e-8, 100, want_log=True)
    print(f"GPU {capi.status_string(res['status'])} K={res['iters']} b^T y={res['dual_obj']!r}; "
          f"oracle {gold['status']} K={gold['iters']} b^T y={gold['dual_obj']!r}", flush=True)
    assert capi.status_string(res["status"]) == "LP_" + gold["status"] == "LP_CONVERGED"
    assert res["iters"] == gold["iters"]
    assert abs(res["dual_obj"] - gold["dual_obj"]) <= 1e-9 * abs(gold["dual_obj"])
    assert abs(res["dual_obj"] - affine["dual_obj"]) <= 1e-9 * abs(affine["dual_obj"])
    x, y, s = (v.cpu().numpy() for v in h.iterate_values())
    assert x @ s < 1e-8 and np.all(x > 0) and np.all(s > 0)


def test_pc_rejects_mixed_and_tape(torch_dev):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(16, 48, 0)
    T = _T(torch, dev, lp)
    for kw in (dict(precision="mixed"), dict(tape_capacity=3)):
        with pytest.raises(RuntimeError, match="LP_ERR_INVALID_ARG"):
            solver.LP(*T, alpha=0.95, method="pc", **kw)
