"""Batched solver (one captured launch sequence per iteration for all LPs)
against the oracle, LP by LP, on ragged shapes m ~ U{16..256}, n = round(r m),
r ~ U(3, 5)."""
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


def _oracle_check(lp, status, iters, x, y, s, strict_iters=True):
    ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
    assert capi.status_string(status) == "LP_" + ro.status_name, (lp.seed, status, ro.status_name)
    if ro.status == oracle.CONVERGED:
        if strict_iters:
            assert iters == ro.iters, (lp.seed, iters, ro.iters)
        byo = lp.b @ ro.y
        assert abs(lp.b @ y - byo) <= 1e-9 * max(1.0, abs(byo)), (lp.seed, lp.b @ y, byo)
        assert x @ s < 1e-8 and np.all(x > 0) and np.all(s > 0)


def test_batch_small_matches_oracle(torch_dev):
    from paper_1502_03543_amd import solver
    lps = lpgen.gen_batch(24, first_seed=100)
    print("shapes:", [lp.A.shape for lp in lps], flush=True)
    bt = solver.Batch(lps, alpha=0.95)
    print("batch set up, solving", flush=True)
    res = bt.solve(1e-8, 200)
    print("solved:", list(res["iters"]), flush=True)
    its = bt.iterates()
    for i, lp in enumerate(lps):
        _oracle_check(lp, res["status"][i], res["iters"][i], *its[i])


def test_batch_mixed_statuses(torch_dev):
    """A zero row gives an exact zero pivot (breakdown) in its LP only; a tight
    iteration limit stops another; the rest converge."""
    from paper_1502_03543_amd import solver
    lps = lpgen.gen_batch(6, first_seed=7)
    bad = lps[2]
    bad.A = bad.A.copy()
    bad.A[min(3, bad.A.shape[0] - 1)] = 0.0
    bad.b = bad.A @ bad.x0
    bt = solver.Batch(lps, alpha=0.95)
    res = bt.solve(1e-8, 200)
    its = bt.iterates()
    assert capi.status_string(res["status"][2]) == "LP_ERR_BREAKDOWN"
    np.testing.assert_array_equal(its[2][0], bad.x0)
    for i, lp in enumerate(lps):
        _oracle_check(lp, res["status"][i], res["iters"][i], *its[i])
    bt2 = solver.Batch(lps[:2], alpha=0.95)
    r2 = bt2.solve(1e-8, 3)
    assert all(capi.status_string(s) == "LP_MAX_ITER" for s in r2["status"])
    assert list(r2["iters"]) == [3, 3]


def test_batch_validation(torch_dev):
    from paper_1502_03543_amd import solver
    lps = lpgen.gen_batch(3, first_seed=1)
    lps[1].s0 = lps[1].s0.copy()
    lps[1].s0[0] = -1.0
    with pytest.raises(RuntimeError, match="LP_ERR_NOT_INTERIOR"):
        solver.Batch(lps)
    lps = lpgen.gen_batch(3, first_seed=1)
    lps[2].c = lps[2].c.copy()
    lps[2].c[1] = np.inf
    with pytest.raises(RuntimeError, match="LP_ERR_INVALID_ARG"):
        solver.Batch(lps)


def test_batch_512_ragged(torch_dev):
    """The 512-LP batch (seeds 0..511): every LP stops with a valid status,
    converged ones satisfy the optimality properties, and a sample of 24 LPs
    matches the oracle one by one."""
    from paper_1502_03543_amd import solver
    lps = lpgen.gen_batch(512, first_seed=0)
    bt = solver.Batch(lps, alpha=0.95)
    print("512 LPs set up, solving", flush=True)
    res = bt.solve(1e-8, 200)
    its = bt.iterates()
    names = [capi.status_string(s) for s in res["status"]]
    print({k: names.count(k) for k in set(names)}, flush=True)
    assert set(names) <= {"LP_CONVERGED", "LP_OPTIMAL_PSI1", "LP_ERR_BREAKDOWN",
                          "LP_ERR_LOST_INTERIOR", "LP_ERR_NONPOS_PSI"}
    assert res["n_converged"] >= 490
    for i, lp in enumerate(lps):
        x, y, s = its[i]
        assert np.all(x > 0) and np.all(s > 0)
        if names[i] == "LP_CONVERGED":
            assert x @ s < 1e-8
            rel = np.linalg.norm(lp.A @ x - lp.b) / np.linalg.norm(lp.b)
            if rel > 1e-7:
                # a late primal-residual floor of its own: compare with the oracle's
                ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
                ref = np.linalg.norm(lp.A @ ro.x - lp.b) / np.linalg.norm(lp.b)
                print(f"LP {i}: primal residual {rel:.1e}, oracle {ref:.1e}", flush=True)
                assert rel <= 10 * ref + 1e-7, (i, rel, ref)
    rng = np.random.default_rng(0)
    for i in rng.choice(512, 24, replace=False):
        _oracle_check(lps[i], res["status"][i], res["iters"][i], *its[i])
