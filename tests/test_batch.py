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


@pytest.mark.parametrize("tile,giters", [(0, 0), (32, 1), (64, 8), (32, 3), (128, 4)])
def test_batch_small_matches_oracle(torch_dev, tile, giters):
    """Every launch choice the autotuner may pick (tile edge 32, 64 or 128,
    iterations per captured graph) against the oracle, LP by LP."""
    from paper_1502_03543_amd import solver
    lps = lpgen.gen_batch(24, first_seed=100)
    print("shapes:", [lp.A.shape for lp in lps], f"tile={tile} graph_iters={giters}", flush=True)
    bt = solver.Batch(lps, alpha=0.95, batch_tile=tile, batch_graph_iters=giters)
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


@pytest.mark.parametrize("launch", ["tuned", "default"])
def test_batch_512_ragged(torch_dev, launch):
    """The 512-LP batch (seeds 0..511): every LP against the oracle's solve of
    that LP, stored by tests/golden/make_golden.py: same status and iteration
    count, b^T y within 1e-9 relative; converged LPs satisfy the optimality
    properties; the 24 largest LPs are also re-solved by the oracle here.
    Both with the launch the bench uses (the autotuner's entry) and with the
    library's default (per-LP tile edges, four iterations per graph)."""
    import json
    import os
    from paper_1502_03543_amd import solver
    with open(os.path.join(os.path.dirname(__file__), "golden", "batch512_seed0.json")) as f:
        gold = json.load(f)["lps"]
    lps = lpgen.gen_batch(512, first_seed=0)
    if launch == "tuned":
        bt = solver.Batch(lps, alpha=0.95)
    else:
        bt = solver.Batch(lps, alpha=0.95, batch_tile=0, batch_graph_iters=0)
    print("512 LPs set up, solving", flush=True)
    res = bt.solve(1e-8, 200)
    its = bt.iterates()
    names = [capi.status_string(s) for s in res["status"]]
    print({k: names.count(k) for k in set(names)}, flush=True)
    n_conv_gold = sum(g["status"] in ("CONVERGED", "OPTIMAL_PSI1") for g in gold)
    assert res["n_converged"] == n_conv_gold, (res["n_converged"], n_conv_gold)
    worst = 0.0
    for i, lp in enumerate(lps):
        g = gold[i]
        assert (g["m"], g["n"], g["seed"]) == (lp.m, lp.n, lp.seed)
        assert names[i] == "LP_" + g["status"], (i, names[i], g["status"])
        x, y, s = its[i]
        assert np.all(x > 0) and np.all(s > 0)
        if g["status"] == "CONVERGED":
            assert res["iters"][i] == g["iters"], (i, res["iters"][i], g["iters"])
            rel = abs(lp.b @ y - g["dual_obj"]) / max(1.0, abs(g["dual_obj"]))
            worst = max(worst, rel)
            assert rel <= 1e-9, (i, lp.b @ y, g["dual_obj"])
            assert x @ s < 1e-8
            rp = np.linalg.norm(lp.A @ x - lp.b) / np.linalg.norm(lp.b)
            assert rp <= 10 * g["primal_residual"] + 1e-7, (i, rp, g["primal_residual"])
    print(f"largest dual-objective difference {worst:.1e}", flush=True)
    big = np.argsort([-(lp.m ** 2 * lp.n) for lp in lps])[:24]
    for i in big:
        _oracle_check(lps[i], res["status"][i], res["iters"][i], *its[i])


def test_batch_iterate_matches_oracle(torch_dev):
    """lp_batch_iterate: one loop pass of every running LP, each step against
    oracle.iterate on that LP's own input iterate (psi, argmax, t, the new
    iterate); an LP stopped by the gap test takes no step."""
    from paper_1502_03543_amd import solver
    lps = lpgen.gen_batch(12, first_seed=300)
    bt = solver.Batch(lps, alpha=0.95)
    print("batch iterate: shapes", [lp.A.shape for lp in lps], flush=True)
    stopped = set()
    for k in range(40):
        its = bt.iterates()
        tol = 1e-8
        st, info = bt.iterate(tol)
        new = bt.iterates()
        for i, lp in enumerate(lps):
            x, y, s = its[i]
            e = info[i]
            if i in stopped:
                assert e["k"] == -1 and e["status"] == st[i] != capi.LP_OK
                continue
            if x @ s < tol:
                assert e["k"] == -1 and capi.status_string(st[i]) == "LP_CONVERGED"
                stopped.add(i)
                continue
            it = oracle.iterate(lp.A, lp.b, lp.c, x, y, s, 0.95)
            assert e["k"] == k, (i, e)
            if it.status != oracle.CONTINUE:
                assert capi.status_string(st[i]) == "LP_" + it.status_name, (i, k, st[i])
                stopped.add(i)
                continue
            kap = np.linalg.cond(it.M)
            tol_dy = max(1e-10, 10 * lp.m * U * kap)
            assert abs(e["psi"] - it.psi) <= tol_dy * it.psi, (i, k, e["psi"], it.psi)
            if abs(e["psi"] - it.psi) <= 1e-14 * it.psi:
                assert e["argmax"] == it.argmax
            assert abs(e["t"] - it.t) <= tol_dy * it.t
            xn, yn, sn = new[i]
            np.testing.assert_allclose(xn, it.x, rtol=0, atol=10 * tol_dy * np.max(np.abs(it.x)))
            np.testing.assert_allclose(yn, it.y, rtol=0,
                                       atol=10 * tol_dy * np.max(np.abs(it.y)) + 1e-12)
            assert abs(e["gap_after"] - it.x @ it.s) <= max(1e-9, 100 * tol_dy) * (it.x @ it.s)
            assert e["min_pivot"] > 0
        if len(stopped) == len(lps):
            break
    assert len(stopped) == len(lps)


def test_batch_mixed_precision_matches_oracle(torch_dev):
    """precision="mixed": every LP against the FP64 oracle (status, K, b^T y
    within 1e-9); early iterations use the FP32 factor (refinement
    converged within refine_max corrections), late ones FP64."""
    from paper_1502_03543_amd import solver
    lps = lpgen.gen_batch(24, first_seed=300)
    bt = solver.Batch(lps, alpha=0.95, precision="mixed")
    used32 = np.zeros(len(lps), dtype=int)
    used64 = np.zeros(len(lps), dtype=int)
    for it in range(200):
        st, info = bt.iterate(1e-8)
        for i, e in enumerate(info):
            if e["k"] < 0:
                continue
            assert 0 <= e["refine_steps"] <= 5
            if e["precision_used"] == capi.LP_PREC_MIXED:
                used32[i] += 1
            else:
                used64[i] += 1
        if not np.any(st == capi.LP_OK):
            break
    print("FP32 iterations per LP:", used32.tolist(), "FP64:", used64.tolist(), flush=True)
    assert used32.sum() > 0 and np.all(used64 > 0)
    its = bt.iterates()
    for i, lp in enumerate(lps):
        _oracle_check(lp, st[i], used32[i] + used64[i], *its[i])


def test_batch_mixed_precision_512(torch_dev):
    """The 512-LP batch in mixed precision against the FP64 oracle's record:
    the same statuses, b^T y within 1e-9 relative for every LP, iteration
    counts equal for all but a few LPs (FP32 rounding may move a late
    iterate across the gap threshold by one step)."""
    import json
    import os
    from paper_1502_03543_amd import solver
    with open(os.path.join(os.path.dirname(__file__), "golden", "batch512_seed0.json")) as f:
        gold = json.load(f)["lps"]
    lps = lpgen.gen_batch(512, first_seed=0)
    bt = solver.Batch(lps, alpha=0.95, precision="mixed")
    res = bt.solve(1e-8, 200)
    its = bt.iterates()
    off = 0
    for i, lp in enumerate(lps):
        g = gold[i]
        assert capi.status_string(res["status"][i]) == "LP_" + g["status"], (i, g["status"])
        x, y, s = its[i]
        assert abs(lp.b @ y - g["dual_obj"]) <= 1e-9 * max(1.0, abs(g["dual_obj"])), i
        off += res["iters"][i] != g["iters"]
    print("LPs whose iteration count differs from FP64:", off, flush=True)
    assert off <= 5
