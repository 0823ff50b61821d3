"""Autotuner for the normal-matrix launch shape (workgroup tile and the split
of the sum over j), measured on the device.

For a shape (m, n) and a precision it times one direction per candidate
(lp_setup with the candidate in lp_options, one lp_iterate with profiling on,
the normal-matrix time from lp_get_timings) and keeps the fastest. Results go
to a JSON cache keyed by device architecture, precision and shape;
``solver.LP`` applies a cached choice when the caller gives none.

    python -m paper_1502_03543_amd.autotune --m 2048 --n 8192 [--precision fp64]
    python -m paper_1502_03543_amd.autotune --batch 512

The batched solver is tuned over its tile edge and the number of
iterations captured per graph, timing whole batched solves; its cache entry
is keyed by the batch's set of shapes and ``solver.Batch`` applies it.

The cache only selects launch parameters of the same kernels; every choice
computes the same normal matrix up to the order of the split-K partial sums.
"""
from __future__ import annotations

import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")

# (0, 0): the library's choice (the stream-K kernel for large shapes)
FP64_CANDIDATES = [(0, 0)] + [(128, s) for s in (1, 2, 3, 4, 6, 8, 12, 16)] + \
                  [(64, s) for s in (1, 2, 4)]
FP32_CANDIDATES = [s for s in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32)]


def _arch() -> str:
    import torch

    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def _key(arch: str, precision: str, m: int, n: int) -> str:
    return f"{arch}/{precision}/m{m}/n{n}"


def load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(precision: str, m: int, n: int, arch: str | None = None) -> dict | None:
    """The cached choice for this shape, or None."""
    cache = load_cache()
    if not cache:
        return None
    if arch is None:
        try:
            arch = _arch()
        except Exception:  # no device: nothing to apply
            return None
    return cache.get(_key(arch, precision, m, n))


def _time_direction(T, precision: str, **cfg) -> float:
    from . import solver

    h = solver.LP(*T, alpha=0.95, precision=precision, profile=True, **cfg)
    h.iterate()
    h.close()
    h = solver.LP(*T, alpha=0.95, precision=precision, profile=True, **cfg)
    h.iterate()
    t = h.timings()
    h.close()
    return t["normal_ms"] / max(t["iterations"], 1)


def tune(m: int, n: int, precision: str = "fp64", seed: int = 0, write: bool = True) -> dict:
    """Time every candidate on a generated LP of shape (m, n); return (and
    optionally cache) the fastest."""
    import numpy as np
    import torch

    from . import capi, lpgen

    capi.load()
    dev = torch.device("cuda:0")
    lp = lpgen.gen_lp(m, n, seed)
    T = [torch.from_numpy(np.ascontiguousarray(v)).to(dev)
         for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
    table = []
    if precision == "fp64":
        for tile, splits in FP64_CANDIDATES:
            ms = _time_direction(T, "fp64", syrk_tile=tile, syrk_splits=splits)
            table.append({"syrk_tile": tile, "syrk_splits": splits, "normal_ms": ms})
    else:
        for splits in FP32_CANDIDATES:
            ms = _time_direction(T, "mixed", syrk32_splits=splits)
            table.append({"syrk32_splits": splits, "normal_ms": ms})
    best = min(table, key=lambda r: r["normal_ms"])
    choice = {k: v for k, v in best.items() if k != "normal_ms"}
    entry = {"choice": choice, "normal_ms": best["normal_ms"], "table": table,
             "measured": time.strftime("%Y-%m-%d")}
    if write:
        cache = load_cache()
        cache[_key(_arch(), precision, m, n)] = entry
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


# batched solver: (batch_tile, batch_graph_iters)
BATCH_CANDIDATES = [(t, g) for t in (0, 64, 32, 128) for g in (1, 2, 4, 8)]


def batch_signature(m, n) -> str:
    """Key of a batch's shape set: count, m range and a digest of the shapes
    (a cached choice applies only to the same set of shapes)."""
    import hashlib

    import numpy as np

    m = np.asarray(m, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    h = hashlib.sha1(m.tobytes() + n.tobytes()).hexdigest()[:12]
    return f"count{len(m)}/m{int(m.min())}-{int(m.max())}/{h}"


def lookup_batch(m, n, arch: str | None = None) -> dict | None:
    """The cached batched launch choice for this set of shapes, or None."""
    cache = load_cache()
    if not cache:
        return None
    if arch is None:
        try:
            arch = _arch()
        except Exception:
            return None
    return cache.get(f"{arch}/batch/fp64/{batch_signature(m, n)}")


def tune_batch(count: int = 512, first_seed: int = 0, reps: int = 2, write: bool = True) -> dict:
    """Time whole batched solves (gap 1e-8, inputs resident, setup excluded)
    of the ragged batch lpgen.gen_batch(count, first_seed) for every
    candidate tile edge and graph length; return (and optionally cache) the
    fastest.  Every candidate computes the same iteration; only the tiling
    of the normal matrices and trailing updates (summation order within a
    tile) and the host-check interval differ."""
    import torch

    from . import capi, lpgen, solver

    capi.load()
    lps = lpgen.gen_batch(count, first_seed=first_seed)
    table = []
    for tile, giters in BATCH_CANDIDATES:
        times = []
        for r in range(reps + 1):
            bt = solver.Batch(lps, alpha=0.95, batch_tile=tile, batch_graph_iters=giters)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = bt.solve(1e-8, 200)
            torch.cuda.synchronize()
            if r > 0:
                times.append(time.perf_counter() - t0)
            bt.close()
        table.append({"batch_tile": tile, "batch_graph_iters": giters,
                      "solve_ms": 1e3 * min(times), "n_converged": int(res["n_converged"])})
        print(json.dumps(table[-1]), flush=True)
    best = min(table, key=lambda r: r["solve_ms"])
    choice = {k: best[k] for k in ("batch_tile", "batch_graph_iters")}
    m = [lp.A.shape[0] for lp in lps]
    n = [lp.A.shape[1] for lp in lps]
    entry = {"choice": choice, "solve_ms": best["solve_ms"], "table": table,
             "workload": f"lpgen.gen_batch({count}, first_seed={first_seed})",
             "measured": time.strftime("%Y-%m-%d")}
    if write:
        cache = load_cache()
        cache[f"{_arch()}/batch/fp64/{batch_signature(m, n)}"] = entry
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--m", type=int)
    ap.add_argument("--n", type=int)
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"))
    ap.add_argument("--batch", type=int, default=0,
                    help="tune the batched solver on lpgen.gen_batch(BATCH) instead")
    args = ap.parse_args()
    if args.batch:
        print(json.dumps(tune_batch(args.batch)))
    else:
        if args.m is None or args.n is None:
            ap.error("--m and --n are required without --batch")
        print(json.dumps(tune(args.m, args.n, args.precision)))


if __name__ == "__main__":
    main()
