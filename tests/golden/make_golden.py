"""Write the oracle-computed fixtures under tests/golden/.

Every value written here comes from the CPU oracle (``oracle/``) run on the
seeded synthetic instances of ``paper_1502_03543_amd.lpgen``; nothing is read
from the GPU library.  The fixtures pin the large configurations whose oracle
runs take minutes, so that the GPU tests can compare against them directly:

  lp64x256_seed0.json          m=64, n=256, seed 0, alpha 0.95, gap 1e-8:
                               status, K, objectives, per-iteration log
  lp2048x8192_seed0.json       m=2048, n=8192, seed 0, alpha 0.95, gap 1e-8:
                               the same, plus the first direction's psi,
                               argmax and t
  lp2048x8192_seed0_dy0.npy    that first direction dy (float64, m)
  lp8192x32768_seed0.json      m=8192, n=32768, seed 0: the first direction
                               from the start point (psi, argmax, t, pivots)
  lp8192x32768_seed0_dy0.npy   its dy (float64, m)
  batch512_seed0.json          512 LPs, seeds 0..511, shapes m ~ U{16..256},
                               n = round(r m), r ~ U(3, 5), alpha 0.95, gap
                               1e-8: per-LP status, K and objectives
  lp2048x8192_seed0_pc.json    the m=2048 instance under the predictor-corrector
                               variant: status, K, objectives, per-iteration log
  lp2048x8192_d01_seed0_csr.json
                               sparse instance (density 1%, seed 0, every row
                               with one guaranteed entry): the same record
                               as lp2048x8192_seed0.json, solved by the
                               oracle on its dense form
  lp2048x8192_d01_seed0_csr_dy0.npy
                               its first direction dy (float64, m)
  fd_lp256x1024_K30.json       64-LP reverse-mode workload (m=256, n=1024,
                               K=30, alpha 0.9, loss w^T x_K): central
                               differences of the loss along seeded directions
                               of A, b and c, in the long-double oracle, at
                               h = 1e-6 and h/2, for a sample of LPs

Usage: python tests/golden/make_golden.py [c1] [c2] [c2pc] [c2sp] [c3] [c4] [c5]
(no argument: all).  The m=2048 solve takes a few minutes on 8 cores, the
m=8192 direction several more.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1502_03543_amd import lpgen  # noqa: E402

FD_LPS = (0, 17, 40)       # LPs of the reverse-mode batch with FD fixtures
FD_H = 1e-6


def fd_direction(key: str, lp_index: int, shape) -> np.ndarray:
    """Seeded test direction for the finite-difference fixture (an input of
    the check, regenerated identically by the test)."""
    salt = {"A": 1, "b": 2, "c": 3}[key]
    E = np.random.default_rng([lp_index, salt, 1502]).standard_normal(shape)
    # unit Frobenius norm: h = 1e-6 then moves the input by 1e-6, so the
    # difference rarely straddles a change of the ratio-test maximiser
    return E / np.linalg.norm(E)


def _dump(name: str, obj) -> None:
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(obj, f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", path, flush=True)


def _solve_record(lp, alpha, tol, max_iter):
    t0 = time.time()
    ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha, tol, max_iter)
    rp = lp.A @ ro.x - lp.b
    rec = dict(
        m=lp.m, n=lp.n, seed=lp.seed, alpha=alpha, gap_tol=tol, max_iter=max_iter,
        status=ro.status_name, iters=ro.iters,
        dual_obj=float(lp.b @ ro.y), primal_obj=float(lp.c @ ro.x),
        gap=float(ro.x @ ro.s),
        primal_residual=float(np.linalg.norm(rp) / np.linalg.norm(lp.b)),
        log=[dict(psi=e["psi"], gap=e["gap"], t=e["t"], argmax=int(e["argmax"]),
                  min_pivot=e["min_pivot"]) for e in ro.log],
        oracle_seconds=round(time.time() - t0, 2), oracle_threads=oracle.num_threads(),
    )
    return rec


def _first_direction(lp, alpha):
    it = oracle.iterate(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha)
    piv = np.diag(it.L) ** 2
    rec = dict(status=it.status_name, psi=it.psi, argmax=int(it.argmax), t=it.t,
               min_pivot=it.min_pivot, max_pivot=float(piv.max()),
               dy_norm=float(np.linalg.norm(it.dy)), gap=it.gap)
    return it, rec


def c1():
    lp = lpgen.gen_lp(64, 256, 0)
    _dump("lp64x256_seed0.json", _solve_record(lp, 0.95, 1e-8, 200))


def c2():
    lp = lpgen.gen_lp(2048, 8192, 0)
    it, first = _first_direction(lp, 0.95)
    np.save(os.path.join(HERE, "lp2048x8192_seed0_dy0.npy"), it.dy)
    del it
    rec = _solve_record(lp, 0.95, 1e-8, 200)
    rec["first_direction"] = first
    _dump("lp2048x8192_seed0.json", rec)


def c2pc():
    """The same m=2048 instance solved by the predictor-corrector oracle."""
    lp = lpgen.gen_lp(2048, 8192, 0)
    t0 = time.time()
    ro = oracle.pc_solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 100)
    rec = dict(m=2048, n=8192, seed=0, eta=0.95, gap_tol=1e-8, status=ro.status_name,
               iters=ro.iters, dual_obj=float(lp.b @ ro.y), primal_obj=float(lp.c @ ro.x),
               gap=float(ro.x @ ro.s), log=ro.log, oracle_seconds=round(time.time() - t0, 2),
               oracle_threads=oracle.num_threads())
    _dump("lp2048x8192_seed0_pc.json", rec)


def c2sp():
    """The sparse m=2048 instance (1% density) solved by the oracle on the
    densified matrix."""
    lp = lpgen.gen_sparse_lp(2048, 8192, 0.01, 0)
    it, first = _first_direction(lp, 0.95)
    np.save(os.path.join(HERE, "lp2048x8192_d01_seed0_csr_dy0.npy"), it.dy)
    del it
    rec = _solve_record(lp, 0.95, 1e-8, 200)
    rec.update(first_direction=first, density=0.01, nnz=lp.nnz)
    _dump("lp2048x8192_d01_seed0_csr.json", rec)


def c3():
    t0 = time.time()
    lp = lpgen.gen_lp(8192, 32768, 0)
    it, rec = _first_direction(lp, 0.95)
    np.save(os.path.join(HERE, "lp8192x32768_seed0_dy0.npy"), it.dy)
    rec.update(m=8192, n=32768, seed=0, alpha=0.95,
               oracle_seconds=round(time.time() - t0, 2), oracle_threads=oracle.num_threads())
    _dump("lp8192x32768_seed0.json", rec)


def c4():
    lps = lpgen.gen_batch(512, first_seed=0)
    out = []
    for i, lp in enumerate(lps):
        r = _solve_record(lp, 0.95, 1e-8, 200)
        del r["log"]
        out.append(r)
        if i % 64 == 0:
            print("LP", i, r["status"], r["iters"], flush=True)
    _dump("batch512_seed0.json", dict(count=512, first_seed=0, lps=out))


def c5():
    m, n, K, alpha = 256, 1024, 30, 0.9
    recs = []
    for i in FD_LPS:
        lp = lpgen.gen_lp(m, n, i)
        w = lpgen.loss_weights(n, i)
        for key, shape in (("A", (m, n)), ("b", (m,)), ("c", (n,))):
            E = fd_direction(key, i, shape)
            vals = {}
            for h in (FD_H, FD_H / 2):
                st_p, lp_p, *_ = oracle.forward_k(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha,
                                                  K, w, {key: E}, h, precision="f80")
                st_m, lp_m, *_ = oracle.forward_k(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, alpha,
                                                  K, w, {key: E}, -h, precision="f80")
                assert st_p == st_m == oracle.CONTINUE, (i, key, st_p, st_m)
                vals[h] = (lp_p - lp_m) / (2 * h)
            recs.append(dict(lp=i, key=key, fd_h=vals[FD_H], fd_h2=vals[FD_H / 2]))
            print(recs[-1], flush=True)
    _dump("fd_lp256x1024_K30.json", dict(m=m, n=n, K=K, alpha=alpha, h=FD_H,
                                         direction="numpy default_rng([lp, salt, 1502]) "
                                                   "standard normal, salt A=1 b=2 c=3, "
                                                   "scaled to unit Frobenius norm",
                                         entries=recs))


if __name__ == "__main__":
    todo = sys.argv[1:] or ["c1", "c2", "c2pc", "c2sp", "c4", "c5", "c3"]
    for name in todo:
        t0 = time.time()
        globals()[name]()
        print(name, "done in %.1f s" % (time.time() - t0), flush=True)
