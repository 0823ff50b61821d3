"""Reverse mode on the GPU (lp_backward, PDASFixedK) against the oracle's
reverse mode on the same problem and against long-double central
differences."""
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


def _T(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


@pytest.mark.parametrize("m,n,K,seed", [(6, 20, 1, 0), (12, 40, 3, 1), (64, 256, 10, 2),
                                        (100, 333, 8, 3)])
def test_backward_matches_oracle(torch_dev, m, n, K, seed):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(m, n, seed)
    w = lpgen.loss_weights(n, seed)
    T = [_T(torch, dev, v) for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
    h = solver.LP(*T, alpha=0.9, tape_capacity=K)
    res = h.solve(0.0, K)
    assert res["status"] == capi.LP_MAX_ITER and res["iters"] == K
    g = h.backward(_T(torch, dev, w))
    # the oracle's reverse mode on the GPU's own recorded trajectory
    st, go = oracle.backward(lp.A, lp.b, lp.c, 0.9, K, h.tape(K), w)
    assert st == oracle.CONTINUE
    # dL/dy0 is exactly zero (x_K does not depend on y0 in the residual form:
    # ds = c - s - A^T M^-1 (b + A D (c - s)) for every y), so it is measured
    # against the largest gradient instead of its own rounding noise
    big = max(np.linalg.norm(go[k]) for k in ("Abar", "bbar", "cbar", "x0bar", "s0bar"))
    for key, okey in (("A", "Abar"), ("b", "bbar"), ("c", "cbar"), ("x0", "x0bar"),
                      ("y0", "y0bar"), ("s0", "s0bar")):
        a = g[key].cpu().numpy()
        o = go[okey]
        scale = max(np.linalg.norm(o), 1e-3 * big)
        rel = np.linalg.norm(a - o) / scale
        print(key, rel)
        assert rel <= 1e-6, (key, rel)


def test_autograd_fd(torch_dev):
    """torch.autograd through PDASFixedK against long-double central
    differences (h = 1e-6) of w^T x_K, K = 2."""
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    m, n, K, seed = 8, 30, 2, 4
    lp = lpgen.gen_lp(m, n, seed)
    w = lpgen.loss_weights(n, seed)
    T = [_T(torch, dev, v).requires_grad_(True) for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
    xK = solver.PDASFixedK.apply(*T, K, 0.9)
    loss = (xK * _T(torch, dev, w)).sum()
    loss.backward()
    rng = np.random.default_rng(0)
    for t, key in zip(T, ("A", "b", "c", "x0", "y0", "s0")):
        E = rng.standard_normal(tuple(t.shape))
        _, lpl, *_ = oracle.forward_k(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.9, K, w,
                                      {key: E}, 1e-6, precision="f80")
        _, lmi, *_ = oracle.forward_k(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.9, K, w,
                                      {key: E}, -1e-6, precision="f80")
        fd = (lpl - lmi) / 2e-6
        an = float((t.grad.cpu().numpy() * E).sum())
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-2), (key, an, fd)


def test_backward_without_tape_fails(torch_dev):
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    lp = lpgen.gen_lp(8, 24, 0)
    T = [_T(torch, dev, v) for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
    h = solver.LP(*T, alpha=0.9)
    h.solve(0.0, 2)
    with pytest.raises(RuntimeError, match="LP_ERR_NO_TAPE"):
        h.backward(_T(torch, dev, np.ones(24)))


def test_batch_backward_differentiable_config(torch_dev):
    """64 LPs, m = 256, n = 1024, K = 30, alpha = 0.9, loss w^T x_K: the batched
    reverse sweep against (1) the oracle's reverse mode on the GPU's own tape
    for 4 LPs, norm-wise, and (2) long-double central differences of the
    forward map (h = 1e-6 and h/2, stored by tests/golden/make_golden.py)
    along seeded directions of A, b and c for 3 LPs.

    Bound: 1e-6 relative, widened to 2 u kappa where the recorded steps'
    normal matrices are worse conditioned than that allows (u the FP64 unit
    roundoff, kappa the largest 2-norm condition number of M over the steps):
    two FP64 evaluations of a solve with M differ by about u kappa, and by
    step 30 kappa reaches 1e10..1e12 (measured errors in the design notes)."""
    import json
    import os
    import sys
    torch, dev = torch_dev
    from paper_1502_03543_amd import solver
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import fd_direction
    with open(os.path.join(os.path.dirname(__file__), "golden", "fd_lp256x1024_K30.json")) as f:
        fdg = json.load(f)
    K = 30
    lps = [lpgen.gen_lp(256, 1024, i) for i in range(64)]
    ws = [lpgen.loss_weights(1024, i) for i in range(64)]
    bt = solver.Batch(lps, alpha=0.9, tape_capacity=K)
    print("64 LPs set up, forward", flush=True)
    res = bt.solve(0.0, K)
    print("forward done, reverse", flush=True)
    assert all(capi.status_string(s) == "LP_MAX_ITER" for s in res["status"]), res["status"]
    assert all(it == K for it in res["iters"])
    g = bt.backward(torch.from_numpy(np.concatenate(ws)).to(dev))
    tapes = bt.tape(K)
    Ag = g["A"].cpu().numpy()
    bg = g["b"].cpu().numpy()
    cg = g["c"].cpu().numpy()

    def grads(i):
        a0 = int(bt.a_off[i])
        return dict(A=Ag[a0:a0 + 256 * 1024].reshape(256, 1024),
                    b=bg[bt.v_off_m[i]:bt.v_off_m[i] + 256],
                    c=cg[bt.v_off_n[i]:bt.v_off_n[i] + 1024])

    fails, kap_of = [], {}
    for i in (0, 17, 40, 63):
        lp = lps[i]
        st, go = oracle.backward(lp.A, lp.b, lp.c, 0.9, K, tapes[i], ws[i])
        assert st == oracle.CONTINUE
        # condition of M at every recorded step (2-norm, from the oracle's M
        # on the GPU's tape row), and the pivot ratio of its factor
        kaps, pivr = [], []
        for r in tapes[i]:
            it = oracle.iterate(lp.A, lp.b, lp.c, r[:1024], r[1024:1280], r[1280:], 0.9)
            kaps.append(np.linalg.cond(it.M))
            piv = np.diag(it.L) ** 2
            pivr.append(piv.max() / piv.min())
        kap = max(kaps)
        kap_of[i] = kap
        gi = grads(i)
        ra = np.linalg.norm(gi["A"] - go["Abar"]) / np.linalg.norm(go["Abar"])
        rb = np.linalg.norm(gi["b"] - go["bbar"]) / np.linalg.norm(go["bbar"])
        rc = np.linalg.norm(gi["c"] - go["cbar"]) / np.linalg.norm(go["cbar"])
        # two FP64 evaluations of the sweep differ by about u kappa(M) per
        # solve with M; the bound takes the worst step
        tol = max(1e-6, 2 * U * kap)
        print(f"LP {i}: Abar {ra:.2e} bbar {rb:.2e} cbar {rc:.2e}; max kappa(M) {kap:.2e} "
              f"(u kappa {U * kap:.1e}, tol {tol:.1e}); pivot ratio max {max(pivr):.1e}",
              flush=True)
        if not (ra <= tol and rb <= tol and rc <= tol):
            fails.append((i, ra, rb, rc, tol))
    h = fdg["h"]
    for e in fdg["entries"]:
        i, key = e["lp"], e["key"]
        E = fd_direction(key, i, grads(i)[key].shape)
        an = float(np.sum(grads(i)[key] * E))
        fd = e["fd_h"]
        # the differences' own spread, and the adjoint's rounding bound
        # 2 u kappa ||grad|| ||E|| (||E|| = 1) projected on the direction
        own = 2 * U * kap_of[i] * np.linalg.norm(grads(i)[key])
        slack = max(1e-6 * abs(an), 2 * abs(e["fd_h"] - e["fd_h2"]), own)
        print(f"FD LP {i} d/d{key}: adjoint {an:.10e} central difference {fd:.10e} "
              f"(h/2: {e['fd_h2']:.10e}) |diff| {abs(an - fd):.1e} allowed {slack:.1e}",
              flush=True)
        if not abs(an - fd) <= slack:
            fails.append((i, key, an, fd, slack))
    assert not fails, fails
