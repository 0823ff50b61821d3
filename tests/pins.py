"""Checks that pin the CPU oracle to facts fixed by the paper and by mathematics,
independent of the oracle's own code.  Each check raises AssertionError on
failure; ``test_oracle_pins.py`` runs them on the real oracle and
``test_oracle_mutants.py`` runs them on deliberately broken copies of it.

Every check takes ``prec``: 'f64', 'f80' or the path of a library built from a
modified copy of the oracle source.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

import oracle
from paper_1502_03543_amd import lpgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lp(m, n, seed):
    return lpgen.gen_lp(m, n, seed)


# ---------------------------------------------------------------- worked example
def check_psi1_example(prec="f64"):
    """Section 3 Algorithm, psi = 1 branch: alpha := 1, full step, stop."""
    g = json.load(open(os.path.join(GOLDEN, "psi1_example.json")))
    e = g["expect"]
    A, b, c = np.array(g["A"]), np.array(g["b"]), np.array(g["c"])
    x0, y0, s0 = np.array(g["x0"]), np.array(g["y0"]), np.array(g["s0"])
    it = oracle.iterate(A, b, c, x0, y0, s0, g["alpha"], precision=prec)
    assert oracle.STATUS_NAMES[it.status] == e["status"], it.status_name
    for k in ("d", "M", "rhs", "dy", "ds", "dx"):
        np.testing.assert_array_equal(getattr(it, k), np.array(e[k]), err_msg=k)
    assert it.psi == e["psi"] and it.argmax == e["argmax"]
    assert it.alpha_eff == e["alpha_eff"] and it.t == e["t"]
    np.testing.assert_array_equal(it.x, e["x1"])
    np.testing.assert_array_equal(it.y, e["y1"])
    np.testing.assert_array_equal(it.s, e["s1"])
    r = oracle.solve(A, b, c, x0, y0, s0, g["alpha"], 1e-8, 50, precision=prec)
    assert r.status_name == e["status"] and r.iters == e["iters"]
    assert c @ r.x == e["primal_obj"] and b @ r.y == e["dual_obj"]


# ---------------------------------------------------------------- Newton system
def _iterates(m, n, seed, prec, alpha=0.95, upto=60):
    lp = _lp(m, n, seed)
    r = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha, 1e-8, upto, tape=True,
                     precision=prec)
    return lp, r


def check_newton_rows(prec="f64", m=12, n=40, seed=3):
    """Section 3, system (bigsystem) with residual right-hand side
    [b - Ax; c - A^T y - s; -Xs]: each block row holds for the direction, and
    row 3 per coordinate gives dx_j/x_j + ds_j/s_j = -1."""
    lp, r = _iterates(m, n, seed, prec)
    assert r.status_name == "CONVERGED", r.status_name
    A = lp.A
    for k in range(0, r.iters, max(1, r.iters // 6)):
        row = r.tape[k]
        x, y, s = row[:n], row[n:n + m], row[n + m:]
        it = oracle.iterate(A, lp.b, lp.c, x, y, s, 0.95, precision=prec)
        dx, dy, ds = it.dx, it.dy, it.ds
        rp = lp.b - A @ x
        rd = lp.c - A.T @ y - s
        scale_p = np.abs(A) @ np.abs(dx) + np.abs(lp.b) + np.abs(A) @ x
        assert np.all(np.abs(A @ dx - rp) <= 1e-9 * scale_p + 1e-300), k
        scale_d = np.abs(A.T) @ np.abs(dy) + np.abs(ds) + np.abs(lp.c) + np.abs(A.T) @ np.abs(y)
        assert np.all(np.abs(A.T @ dy + ds - rd) <= 1e-12 * scale_d), k
        assert np.all(np.abs(s * dx + x * ds + x * s) <= 1e-12 * (np.abs(s * dx) + np.abs(x * ds) + x * s)), k
        np.testing.assert_allclose(dx / x + ds / s, -1.0, rtol=0, atol=1e-10)
        # recorded residual vectors are the definitions
        np.testing.assert_allclose(it.r_d, rd, rtol=0, atol=1e-12 * np.max(np.abs(lp.c)))
        np.testing.assert_allclose(it.d, x / s, rtol=1e-15)


def check_gap_identity(prec="f64", m=10, n=30, seed=5):
    """After the step (x,s) += t(dx,ds): x+_j s+_j = (1-t) x_j s_j + t^2 dx_j ds_j
    (row 3 of the Newton system), and with feasibility dx^T ds = 0 so
    gap+ = (1 - alpha/psi) gap (Section 3 update rule)."""
    lp, r = _iterates(m, n, seed, prec)
    for k in range(r.iters):
        row = r.tape[k]
        x, y, s = row[:n], row[n:n + m], row[n + m:]
        it = oracle.iterate(lp.A, lp.b, lp.c, x, y, s, 0.95, precision=prec)
        t = it.t
        lhs = it.x * it.s
        rhs = (1 - t) * x * s + t * t * it.dx * it.ds
        np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-14 * np.max(x * s))
        gap = x @ s
        assert abs(it.dx @ it.ds) <= 1e-7 * max(gap, 1e-300) + 1e-12 * np.abs(it.dx) @ np.abs(it.ds)
        assert it.psi >= 1 - 1e-9, it.psi
        np.testing.assert_allclose(it.x @ it.s, (1 - 0.95 / it.psi) * gap, rtol=1e-6,
                                   atol=1e-13 * np.abs(it.dx) @ np.abs(it.ds))
        # Algorithm step length and ratio test, by definition
        u = np.concatenate([-it.dx / x, -it.ds / s])
        assert it.psi == np.max(u) and it.argmax == int(np.argmax(u))
        assert it.t == 0.95 / it.psi
        # positivity after a step with alpha < 1
        assert np.all(it.x > 0) and np.all(it.s > 0)


# ---------------------------------------------------------------- closed forms
def check_m1_closed_form(prec="f64", n=9, seed=2):
    """m = 1: M = sum_j d_j a_j^2 and dy = rhs / M (Section 5 normal equations)."""
    lp = _lp(1, n, seed)
    it = oracle.iterate(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.9, precision=prec)
    a = lp.A[0]
    d = lp.x0 / lp.s0
    Mv = np.sum(d * a * a)
    np.testing.assert_allclose(it.M[0, 0], Mv, rtol=1e-14)
    rd = lp.c - a * lp.y0[0] - lp.s0
    rhs = lp.b[0] + np.sum(a * d * rd)
    np.testing.assert_allclose(it.dy[0], rhs / Mv, rtol=1e-13)


def check_normal_matrix_and_cholesky(prec="f64", m=16, n=50, seed=7):
    """M = A D A^T is symmetric positive definite and M v = A (d o (A^T v));
    the factor is lower triangular with positive diagonal and L L^T = M; the
    solve satisfies M w = r to backward-stable accuracy."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    d = rng.uniform(0.1, 10, n)
    M = oracle.normal_matrix(A, d, precision=prec)
    assert np.array_equal(M, M.T)
    v = rng.standard_normal(m)
    bound = 1e-12 * (np.abs(A) @ (d * (np.abs(A.T) @ np.abs(v))))
    assert np.all(np.abs(M @ v - A @ (d * (A.T @ v))) <= bound)
    L, fail, minp = oracle.cholesky(M, precision=prec)
    assert fail == -1
    assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) > 0)
    np.testing.assert_allclose(L @ L.T, M, rtol=0, atol=1e-13 * np.max(np.abs(M)))
    assert abs(minp - np.min(np.diag(L)) ** 2) <= 1e-12 * minp
    r = rng.standard_normal(m)
    w = oracle.cholesky_solve(L, r, precision=prec)
    res = np.linalg.norm(M @ w - r) / (np.linalg.norm(M, 2) * np.linalg.norm(w))
    assert res < 100 * m * 2.0 ** -53, res


def check_cholesky_breakdown(prec="f64", n=20, seed=1):
    """Duplicate rows make A D A^T singular: the factorisation must report a
    non-positive pivot, not return numbers."""
    lp = _lp(4, n, seed)
    A = lp.A.copy()
    A[3] = A[1]
    b = A @ lp.x0
    it = oracle.iterate(A, b, lp.c, lp.x0, lp.y0, lp.s0, 0.9, precision=prec)
    assert it.status_name == "ERR_BREAKDOWN", it.status_name
    assert it.fail_col == 3


# ---------------------------------------------------------------- independent solver
def check_egidi_maponi(prec="f64", m=6, n=20, seed=11):
    """Section 5: the Sherman-Morrison recurrence over the split
    ADA^T = AA^T + sum_l (d_l - 1) a_l a_l^T reproduces dy = (ADA^T)^-1 rhs.
    Readings: x_0 = (AA^T)^-1 rhs, v_l = (d_l - 1) a_l (the garbled D_ii is D_jj)."""
    lp = _lp(m, n, seed)
    it = oracle.iterate(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.9, precision=prec)
    A, d = lp.A, it.d
    G = A @ A.T
    Y = np.linalg.solve(G, A)          # columns y_{0,k} = (AA^T)^-1 a_k
    xv = np.linalg.solve(G, it.rhs)    # x_0
    for l in range(n):
        v = (d[l] - 1.0) * A[:, l]
        yl = Y[:, l].copy()
        den = 1.0 + v @ yl
        xv = xv - (v @ xv) / den * yl
        if l + 1 < n:
            Y[:, l + 1:] -= np.outer(yl, (v @ Y[:, l + 1:]) / den)
    np.testing.assert_allclose(it.dy, xv, rtol=1e-9, atol=1e-12 * np.max(np.abs(xv)))


# ---------------------------------------------------------------- vertices
def _vertex_optimum(A, b, c):
    m, n = A.shape
    best = np.inf
    for B in itertools.combinations(range(n), m):
        AB = A[:, B]
        if abs(np.linalg.det(AB)) < 1e-12:
            continue
        xB = np.linalg.solve(AB, b)
        if np.all(xB >= -1e-12):
            best = min(best, c[list(B)] @ xB)
    return best


def check_vertex_enumeration(prec="f64", seeds=(0, 1, 2, 3), m=3, n=8):
    """Section 2: the optimum sits at a vertex.  Enumerating every basis gives
    z*; the final iterate must bracket it by weak duality."""
    for seed in seeds:
        lp = _lp(m, n, seed)
        z = _vertex_optimum(lp.A, lp.b, lp.c)
        r = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-10, 200, precision=prec)
        assert r.status_name in ("CONVERGED", "OPTIMAL_PSI1"), (seed, r.status_name)
        gap = r.x @ r.s
        by, cx = lp.b @ r.y, lp.c @ r.x
        rp = np.linalg.norm(lp.A @ r.x - lp.b)
        assert by <= z + 1e-9 * max(1, abs(z)), (seed, by, z)
        assert cx - z <= gap + np.linalg.norm(r.y) * rp + 1e-9 * max(1, abs(z)), (seed, cx, z)
        assert abs(by - z) <= 1e-8 * max(1, abs(z)), (seed, by, z)
        assert np.all(r.x > 0) and np.all(r.s > 0)


def check_invariants_final(prec="f64", m=64, n=256, seeds=(0, 1)):
    """Converged iterate: Ax = b, A^T y + s = c, c^T x - b^T y = x^T s (exact
    identity for feasible points), x, s > 0 and gap below tolerance."""
    for seed in seeds:
        lp = _lp(m, n, seed)
        r = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200, precision=prec)
        assert r.status_name == "CONVERGED", r.status_name
        x, y, s = r.x, r.y, r.s
        assert x @ s < 1e-8
        assert np.linalg.norm(lp.A @ x - lp.b) <= 1e-9 * np.linalg.norm(lp.b)
        assert np.linalg.norm(lp.A.T @ y + s - lp.c) <= 1e-12 * np.linalg.norm(lp.c)
        assert abs((lp.c @ x - lp.b @ y) - x @ s) <= 1e-9 * max(1.0, abs(lp.c @ x))
        assert np.all(x > 0) and np.all(s > 0)


# ---------------------------------------------------------------- derivatives
def check_adjoint_fd(prec="f64", m=5, n=16, seed=4, Ks=(1, 2, 3), alpha=0.9):
    """Reverse mode against central differences computed with the long-double
    forward (h = 1e-6), for random directions in A, b, c, x0, y0, s0."""
    lp = _lp(m, n, seed)
    w = lpgen.loss_weights(n, seed)
    rng = np.random.default_rng(100 + seed)
    for K in Ks:
        r = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha, 0.0, K, tape=True,
                         precision=prec)
        assert r.iters == K
        st, g = oracle.backward(lp.A, lp.b, lp.c, alpha, K, r.tape, w, precision=prec)
        assert st == oracle.CONTINUE, st
        pairs = []
        for key, gkey, shape in (("A", "Abar", (m, n)), ("b", "bbar", (m,)), ("c", "cbar", (n,)),
                                 ("x0", "x0bar", (n,)), ("y0", "y0bar", (m,)),
                                 ("s0", "s0bar", (n,))):
            E = rng.standard_normal(shape)
            h = 1e-6
            _, lp_, *_ = oracle.forward_k(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha, K, w,
                                          {key: E}, h, precision="f80")
            _, lm_, *_ = oracle.forward_k(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha, K, w,
                                          {key: E}, -h, precision="f80")
            pairs.append((key, float(np.sum(g[gkey] * E)), (lp_ - lm_) / (2 * h)))
        scale = max(abs(fd) for _, _, fd in pairs)
        for key, an, fd in pairs:
            # some derivatives vanish exactly (a y0 shift stays in range(A^T) and is
            # projected out of dx), so the floor is relative to the largest one
            assert abs(an - fd) <= 1e-7 * max(abs(fd), 1e-3 * scale), (K, key, an, fd)


def check_jvp_vjp(prec="f64", m=6, n=20, seed=9, K=4, alpha=0.9):
    """Dot-product identity <VJP(w), v> = <w, JVP(v)> between the independently
    derived forward and reverse modes."""
    lp = _lp(m, n, seed)
    w = lpgen.loss_weights(n, seed)
    rng = np.random.default_rng(seed)
    r = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha, 0.0, K, tape=True,
                     precision=prec)
    st, g = oracle.backward(lp.A, lp.b, lp.c, alpha, K, r.tape, w, precision=prec)
    tang = dict(A=rng.standard_normal((m, n)), b=rng.standard_normal(m),
                c=rng.standard_normal(n), x0=rng.standard_normal(n),
                y0=rng.standard_normal(m), s0=rng.standard_normal(n))
    st2, tx, ty, ts = oracle.jvp(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha, K, tang,
                                 precision=prec)
    lhs = sum(float(np.sum(g[k + "bar"] * tang[k])) for k in tang)
    rhs = float(w @ tx)
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs)), (lhs, rhs)


# ---------------------------------------------------------------- predictor-corrector
def _pc_trajectory(m, n, seed, prec, eta=0.95, upto=60):
    """Start iterate of every predictor-corrector step of one LP."""
    lp = _lp(m, n, seed)
    x, y, s = lp.x0.copy(), lp.y0.copy(), lp.s0.copy()
    out = []
    for _ in range(upto):
        if x @ s < 1e-8:
            break
        r = oracle.pc_iterate(lp.A, lp.b, lp.c, x, y, s, eta, precision=prec)
        out.append(((x, y, s), r))
        if r.status != oracle.CONTINUE:
            break
        x, y, s = r.x, r.y, r.s
    return lp, out


def _kkt_solve(A, x, s, rp, rd, rc):
    """The full Newton system (bigsystem) of the Section 3 algorithm,
    unreduced: [A 0 0; 0 A^T I; S 0 X] [dx; dy; ds] = [rp; rd; rc], solved
    densely by a library routine (test-only, independent of the oracle's
    Section 5 reduction and Cholesky)."""
    m, n = A.shape
    K = np.zeros((m + 2 * n, 2 * n + m))
    K[:m, :n] = A
    K[m:m + n, n:n + m] = A.T
    K[m:m + n, n + m:] = np.eye(n)
    K[m + n:, :n] = np.diag(s)
    K[m + n:, n + m:] = np.diag(x)
    v = np.linalg.solve(K, np.concatenate([rp, rd, rc]))
    return v[:n], v[n:n + m], v[n + m:]


def check_pc_newton_systems(prec="f64", m=6, n=18, seed=12):
    """Predictor-corrector (the Mehrotra method cited in the previous-work
    section): both directions solve the unreduced Newton system, the
    predictor with third right-hand side -Xs and the corrector with
    -Xs - dx_aff o ds_aff + sigma mu e (sigma, mu and the predictor as the
    oracle reports them).  Catches sign and dropped-term errors in the
    reduction of either right-hand side."""
    lp, traj = _pc_trajectory(m, n, seed, prec)
    assert traj and traj[-1][1].status_name in ("CONTINUE",), traj[-1][1].status_name
    for k, ((x, y, s), r) in enumerate(traj[:8]):
        A = lp.A
        rp, rd = lp.b - A @ x, lp.c - A.T @ y - s
        dxa, dya, dsa = _kkt_solve(A, x, s, rp, rd, -x * s)
        sc = lambda v: 1e-9 * max(1.0, np.max(np.abs(v)))
        np.testing.assert_allclose(r.dx_aff, dxa, rtol=0, atol=sc(dxa), err_msg=f"dx_aff {k}")
        np.testing.assert_allclose(r.dy_aff, dya, rtol=0, atol=sc(dya), err_msg=f"dy_aff {k}")
        np.testing.assert_allclose(r.ds_aff, dsa, rtol=0, atol=sc(dsa), err_msg=f"ds_aff {k}")
        rc = -x * s - r.dx_aff * r.ds_aff + r.sigma * r.mu
        dx, dy, ds = _kkt_solve(A, x, s, rp, rd, rc)
        np.testing.assert_allclose(r.dx, dx, rtol=0, atol=sc(dx), err_msg=f"dx {k}")
        np.testing.assert_allclose(r.dy, dy, rtol=0, atol=sc(dy), err_msg=f"dy {k}")
        np.testing.assert_allclose(r.ds, ds, rtol=0, atol=sc(ds), err_msg=f"ds {k}")


def check_pc_steps(prec="f64", m=8, n=30, seed=13, eta=0.95):
    """Predictor-corrector step lengths: each is the largest step keeping the
    iterate non-negative (capped at 1; the corrector's scaled by eta), so the
    predictor step reaches the boundary exactly when below 1, the corrector
    step stops a fraction 1 - eta short of it; the iterate moves by
    alpha_p (dx) and alpha_d (dy, ds); mu is the mean complementarity."""
    lp, traj = _pc_trajectory(m, n, seed, prec, eta)
    assert len(traj) >= 5
    for k, ((x, y, s), r) in enumerate(traj):
        if r.status != oracle.CONTINUE:
            break
        assert abs(r.mu - (x @ s) / n) <= 1e-14 * r.mu
        for v, dv, a, cap in ((x, r.dx_aff, r.alpha_aff_p, 1.0), (s, r.ds_aff, r.alpha_aff_d, 1.0)):
            w = v + a * dv
            assert 0 < a <= cap and np.all(w >= -1e-14 * np.max(v)), (k, a)
            if a < cap:
                assert np.min(w / v) <= 1e-12, (k, a, np.min(w / v))
        for v, dv, a in ((x, r.dx, r.alpha_p), (s, r.ds, r.alpha_d)):
            assert 0 < a <= 1
            if a < 1:
                # a / eta reaches the boundary
                w = v + (a / eta) * dv
                assert abs(np.min(w / v)) <= 1e-12, (k, a, np.min(w / v))
        np.testing.assert_allclose(r.x, x + r.alpha_p * r.dx, rtol=1e-15, atol=0)
        np.testing.assert_allclose(r.y, y + r.alpha_d * r.dy, rtol=1e-15,
                                   atol=1e-15 * np.max(np.abs(y)))
        np.testing.assert_allclose(r.s, s + r.alpha_d * r.ds, rtol=1e-15, atol=0)
        assert np.all(r.x > 0) and np.all(r.s > 0)
        assert 0 <= r.sigma <= 1.0 + 1e-12, (k, r.sigma)


def check_pc_optimum(prec="f64", seeds=(0, 1, 2), m=3, n=8):
    """The predictor-corrector loop ends at the LP optimum that vertex
    enumeration gives (Section 2), and at m=64, n=256 at the Section 3
    algorithm's dual objective, in fewer iterations."""
    for seed in seeds:
        lp = _lp(m, n, seed)
        z = _vertex_optimum(lp.A, lp.b, lp.c)
        r = oracle.pc_solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-10, 100,
                            precision=prec)
        assert r.status_name == "CONVERGED", (seed, r.status_name)
        assert abs(lp.b @ r.y - z) <= 1e-8 * max(1, abs(z)), (seed, lp.b @ r.y, z)
    lp = _lp(64, 256, 0)
    r = oracle.pc_solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 100, precision=prec)
    a = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200, precision=prec)
    assert r.status_name == a.status_name == "CONVERGED"
    assert abs(lp.b @ r.y - lp.b @ a.y) <= 1e-9 * abs(lp.b @ a.y)
    assert r.iters < a.iters, (r.iters, a.iters)
    assert np.linalg.norm(lp.A @ r.x - lp.b) <= 1e-9 * np.linalg.norm(lp.b)


ALL_CHECKS = [
    check_psi1_example, check_newton_rows, check_gap_identity, check_m1_closed_form,
    check_normal_matrix_and_cholesky, check_cholesky_breakdown, check_egidi_maponi,
    check_vertex_enumeration, check_invariants_final, check_adjoint_fd, check_jvp_vjp,
    check_pc_newton_systems, check_pc_steps, check_pc_optimum,
]
