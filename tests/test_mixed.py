"""Mixed precision (FP32 normal matrix and factor, FP64 refinement) against the
FP64 oracle and the FP64 GPU path.

The reference for every mixed-precision direction is FP64: the oracle at sizes
it finishes in seconds, the (oracle-checked) FP64 GPU path at m = 8192.
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


def _T(torch, dev, lp):
    return [torch.from_numpy(np.ascontiguousarray(v)).to(dev)
            for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]


@pytest.mark.parametrize("m,n,seed", [(256, 1024, 0), (300, 1000, 1), (512, 2048, 2)])
def test_mixed_per_iteration_error(torch_dev, m, n, seed):
    """Each mixed step, on the GPU's own input iterate, against the FP64 oracle
    direction; the FP32 factor is used early and FP64 takes over for good."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(m, n, seed)
    print(f"mixed per-iteration m={m} n={n} seed={seed}", flush=True)
    h = solver.LP(*_T(torch, dev, lp), alpha=0.95, precision="mixed")
    precs, errs = [], []
    for k in range(80):
        x, y, s = (v.cpu().numpy() for v in h.iterate_values())
        if x @ s < 1e-8:
            break
        info = h.iterate()
        assert info["status"] == capi.LP_OK, capi.status_string(info["status"])
        _, dyg, _ = (v.cpu().numpy() for v in h.direction())
        it = oracle.iterate(lp.A, lp.b, lp.c, x, y, s, 0.95)
        kap = np.linalg.cond(it.M)
        rel = np.linalg.norm(dyg - it.dy) / np.linalg.norm(it.dy)
        precs.append(info["precision_used"])
        errs.append(rel)
        assert rel <= max(1e-10, 10 * m * U * kap), (k, rel, kap, info)
        if info["precision_used"] == capi.LP_PREC_MIXED:
            assert info["refine_resid"] <= 2.0 ** -46 and info["refine_steps"] >= 1
            assert info["gap_before"] >= 1e-6
    print("precision per iteration:", precs)
    print("dy relative error per iteration:", ["%.1e" % e for e in errs])
    assert precs[0] == capi.LP_PREC_MIXED
    # once FP64 takes over it stays
    first64 = precs.index(capi.LP_PREC_FP64) if capi.LP_PREC_FP64 in precs else len(precs)
    assert all(p == capi.LP_PREC_FP64 for p in precs[first64:])


@pytest.mark.parametrize("m,n,seed", [(256, 1024, 3), (400, 1600, 4)])
def test_mixed_solve_matches_oracle(torch_dev, m, n, seed):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(m, n, seed)
    h = solver.LP(*_T(torch, dev, lp), alpha=0.95, precision="mixed")
    res = h.solve(1e-8, 200)
    ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
    assert capi.status_string(res["status"]) == "LP_" + ro.status_name
    if ro.status == oracle.CONVERGED:
        assert abs(res["iters"] - ro.iters) <= 1
        byo = lp.b @ ro.y
        assert abs(res["dual_obj"] - byo) <= 1e-9 * max(1.0, abs(byo))
        x, y, s = (v.cpu().numpy() for v in h.iterate_values())
        assert x @ s < 1e-8 and np.all(x > 0) and np.all(s > 0)


def test_forced_fallback_is_fp64(torch_dev):
    """refine_max = 0 with a zero tolerance makes every FP32 attempt fall back
    on the first iteration; from then on the path is the FP64 one, bit for bit."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(200, 700, 6)
    T = _T(torch, dev, lp)
    hm = solver.LP(*T, alpha=0.95, precision="mixed", refine_tol=0.0, refine_max=0)
    hf = solver.LP(*T, alpha=0.95)
    for k in range(10):
        im, if_ = hm.iterate(), hf.iterate()
        assert im["precision_used"] == capi.LP_PREC_FP64
        assert im["status"] == if_["status"] == capi.LP_OK
        for a, b in zip(hm.iterate_values(), hf.iterate_values()):
            assert torch.equal(a, b), k


def test_full_size_mixed_lp8192x32768(torch_dev):
    """m = 8192, n = 32768, seed 0: the first direction of the mixed and of the
    FP64 path against the oracle's (tests/golden/make_golden.py) within 1e-10;
    both solves converge to the same dual objective."""
    import json
    import os
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    with open(os.path.join(gdir, "lp8192x32768_seed0.json")) as f:
        gold = json.load(f)
    dy0 = torch.from_numpy(np.load(os.path.join(gdir, "lp8192x32768_seed0_dy0.npy"))).to(dev)
    m, n = 8192, 32768
    print("generating the m=8192 n=32768 instance", flush=True)
    lp = lpgen.gen_lp(m, n, 0)
    T = _T(torch, dev, lp)
    del lp.A
    hm = solver.LP(*T, alpha=0.95, precision="mixed")
    hf = solver.LP(*T, alpha=0.95)
    i_m, i_f = hm.iterate(), hf.iterate()
    assert i_m["precision_used"] == capi.LP_PREC_MIXED and i_m["status"] == capi.LP_OK
    _, dym, _ = hm.direction()
    _, dyf, _ = hf.direction()
    nrm = float(torch.linalg.norm(dy0))
    rel_m = float(torch.linalg.norm(dym - dy0)) / nrm
    rel_f = float(torch.linalg.norm(dyf - dy0)) / nrm
    print(f"first direction vs the FP64 oracle: mixed {rel_m:.2e} "
          f"(refinement steps {i_m['refine_steps']}), FP64 {rel_f:.2e}", flush=True)
    assert rel_f <= 1e-10 and rel_m <= 1e-10
    for info in (i_m, i_f):
        assert abs(info["psi"] - gold["psi"]) <= 1e-10 * gold["psi"]
        assert info["argmax"] == gold["argmax"]
    print("mixed solve", flush=True)
    rm = hm.solve(1e-8, 300, want_log=True)
    print("fp64 solve", flush=True)
    rf = hf.solve(1e-8, 300)
    assert rm["status"] == rf["status"] == capi.LP_CONVERGED
    nmix = sum(1 for e in rm["log"] if e["precision_used"] == capi.LP_PREC_MIXED)
    print(f"iterations mixed {rm['iters'] + 1} (FP32 factor in {nmix + 1}), fp64 {rf['iters'] + 1}")
    assert abs(rm["dual_obj"] - rf["dual_obj"]) <= 1e-9 * max(1.0, abs(rf["dual_obj"]))
    x, y, s = hm.iterate_values()
    assert float(x @ s) < 1e-8 and bool((x > 0).all()) and bool((s > 0).all())
