"""Autotuner for the normal-matrix launch shape (workgroup tile and the split
of the sum over j), measured on the device.

For a shape (m, n) and a precision it times one direction per candidate
(lp_setup with the candidate in lp_options, one lp_iterate with profiling on,
the normal-matrix time from lp_get_timings) and keeps the fastest. Results go
to a JSON cache keyed by device architecture, precision and shape;
``solver.LP`` applies a cached choice when the caller gives none.

    python -m paper_1502_03543_amd.autotune --m 2048 --n 8192 [--precision fp64]

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--m", type=int, required=True)
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"))
    args = ap.parse_args()
    print(json.dumps(tune(args.m, args.n, args.precision)))


if __name__ == "__main__":
    main()
