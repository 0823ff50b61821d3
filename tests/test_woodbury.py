"""The paper's Section 5 direction solver on the GPU (lp_options.solver =
LP_SOLVER_WOODBURY: A A^T factored once, then the Egidi-Maponi rank-one
recurrence per iteration) against the oracle, whose direction is the plain
definition dy = (A D A^T)^-1 rhs (Cholesky): every step on the GPU's own input
iterate within max(1e-10, 10 m u kappa(M)), and whole solves with the same
status, K and b^T y within 1e-9 relative.  (The recurrence itself is pinned
to that definition on the CPU by tests/pins.py::check_egidi_maponi.)"""
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


@pytest.mark.parametrize("m,n,seed", [(64, 256, 0), (64, 256, 1), (37, 150, 4)])
def test_woodbury_iteration_parity(torch_dev, m, n, seed):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(m, n, seed)
    print(f"woodbury iteration parity m={m} n={n} seed={seed}", flush=True)
    h = solver.LP(*_T(torch, dev, lp), alpha=0.95, solver="woodbury")
    steps, worst = 0, 0.0
    for k in range(80):
        x, y, s = (v.cpu().numpy() for v in h.iterate_values())
        if x @ s < 1e-8:
            break
        info = h.iterate()
        it = oracle.iterate(lp.A, lp.b, lp.c, x, y, s, 0.95)
        assert info["status"] == capi.LP_OK and it.status == oracle.CONTINUE, (k, info, it.status)
        _, dyg, _ = (v.cpu().numpy() for v in h.direction())
        kap = np.linalg.cond(it.M)
        tol = max(1e-10, 10 * m * U * kap)
        rel = np.linalg.norm(dyg - it.dy) / np.linalg.norm(it.dy)
        worst = max(worst, rel / (10 * m * U * kap))
        print(f"k={k} kappa {kap:.1e} dy rel {rel:.1e} (bound {tol:.1e})", flush=True)
        assert rel <= tol, (k, rel, tol, kap)
        # psi and the new iterate follow from dy: a difference e in dy moves
        # ds by A^T e and dx by d o A^T e, so each ratio -ds_j/s_j, -dx_j/x_j
        # by at most |A^T e|_j / s_j (late in the run s_j is tiny for the
        # basic columns, where this dominates the dy bound)
        dd = np.abs(lp.A.T @ (dyg - it.dy))
        psi_bound = tol * it.psi + 2 * np.max(dd / s)
        assert abs(info["psi"] - it.psi) <= psi_bound, (k, info["psi"], it.psi, psi_bound)
        if abs(info["psi"] - it.psi) <= 1e-14 * it.psi:
            assert info["argmax"] == it.argmax
        assert info["min_pivot"] > 0
        xn, yn, sn = (v.cpu().numpy() for v in h.iterate_values())
        dt = abs(info["t"] - it.t)
        ex = dt * np.abs(it.dx) + info["t"] * it.d * dd
        ey = dt * np.abs(it.dy) + info["t"] * np.abs(dyg - it.dy)
        assert np.all(np.abs(xn - it.x) <= 2 * ex + 10 * tol * np.max(np.abs(it.x))), k
        assert np.all(np.abs(yn - it.y) <= 2 * ey + 10 * tol * np.max(np.abs(it.y)) + 1e-12), k
        steps += 1
    print(f"{steps} steps; largest dy difference / bound {worst:.2e}", flush=True)
    assert steps >= 10


@pytest.mark.parametrize("m,n,seed", [(64, 256, 0), (64, 256, 1), (64, 256, 2), (37, 150, 4),
                                      (90, 180, 5)])
def test_woodbury_solve_parity(torch_dev, m, n, seed):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(m, n, seed)
    h = solver.LP(*_T(torch, dev, lp), alpha=0.95, solver="woodbury")
    res = h.solve(1e-8, 200)
    ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
    print(f"m={m} n={n} seed={seed}: GPU {capi.status_string(res['status'])} K={res['iters']}; "
          f"oracle {ro.status_name} K={ro.iters}", flush=True)
    assert capi.status_string(res["status"]) == "LP_" + ro.status_name
    if ro.status == oracle.CONVERGED:
        assert res["iters"] == ro.iters
        byo = lp.b @ ro.y
        assert abs(res["dual_obj"] - byo) <= 1e-9 * max(1.0, abs(byo))
        x, y, s = (v.cpu().numpy() for v in h.iterate_values())
        assert x @ s < 1e-8 and np.all(x > 0) and np.all(s > 0)


def test_woodbury_rank_deficient_and_limits(torch_dev):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(16, 48, 0)
    lp.A = lp.A.copy()
    lp.A[5] = 0.0
    lp.b = lp.A @ lp.x0
    with pytest.raises(RuntimeError, match="LP_ERR_BREAKDOWN"):
        solver.LP(*_T(torch, dev, lp), alpha=0.95, solver="woodbury")
    big = lpgen.gen_lp(128, 1024, 0)
    with pytest.raises(RuntimeError, match="LP_ERR_SHAPE"):
        solver.LP(*_T(torch, dev, big), alpha=0.95, solver="woodbury")
