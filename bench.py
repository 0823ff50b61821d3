"""Benchmark: Primal-Dual Affine Scaling solves on one MI355X.

A step is one whole LP solve (the Section 3 loop to x^T s < 1e-8: normal
matrix, Cholesky, triangular solves, direction, ratio test and step in every
iteration) of the m=2048, n=8192 FP64 instance from the Gaussian
interior-feasible generator (seed 0, alpha 0.95).  Inputs and handles are
set up in HBM before the timed region; each step solves a fresh handle from
the same start point.

Prints one JSON line: LP solves/s, plus the normal-matrix kernel's roofline
(FP64 MFMA), the GFLOP/s of normal matrix + Cholesky, and the CPU oracle
timed on a bounded sample of the same workload.

The same line carries the batched comparison (512 ragged LPs solved together
against the single-LP FP64 solver applied LP by LP on a sample of them), the
reverse-mode workload (64 LPs, K = 30 steps with a tape plus the reverse
sweep, with the oracle's forward and reverse sweep on a sample beside it) and
the mixed-precision comparison (m=8192, n=32768: one mixed solve against one
FP64 solve, with the FP64 Cholesky and the FP32 and FP64 normal-matrix
kernels against their peaks), the predictor-corrector variant (Mehrotra's
method, cited in the paper's previous work) on the main instance, and the
paper's own Woodbury / Egidi-Maponi direction solver at m=64, n=256 beside the
Cholesky path.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-variants]
  python bench.py --mixed-compare   # m=8192, n=32768: mixed precision vs FP64, one solve each
  python bench.py --copy-probe      # plain 256 MiB copies (counter scaling)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "lp2048x8192": dict(m=2048, n=8192, seed=0, alpha=0.95, tol=1e-8,
                        desc="single LP m=2048 n=8192 FP64, Gaussian A, alpha 0.95, to gap 1e-8"),
    "lp8192x32768": dict(m=8192, n=32768, seed=0, alpha=0.95, tol=1e-8,
                         desc="single LP m=8192 n=32768 FP64, Gaussian A, alpha 0.95, to gap 1e-8"),
    "lp64x256": dict(m=64, n=256, seed=0, alpha=0.95, tol=1e-8,
                     desc="single LP m=64 n=256 FP64, Gaussian A, alpha 0.95, to gap 1e-8"),
}


def syrk_flops(m: int, n: int) -> float:
    return float(m) * (m + 1) * n


def potrf_flops(m: int) -> float:
    return m ** 3 / 3.0 + m ** 2 / 2.0 + m / 6.0


def source_digest() -> str:
    """Digest of the normal-matrix kernel sources with comments and blank
    lines dropped (a comment edit does not invalidate measured counters)."""
    h = hashlib.sha256()
    for name in ("kernels_syrk.hip", "syrk_tile.h"):
        p = os.path.join(ROOT, "paper_1502_03543_amd", "csrc", name)
        for line in open(p):
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def read_traffic(m: int, n: int):
    """HBM bytes per normal-matrix kernel launch from the committed counter
    summary, or None when absent or measured on a different kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic_normal_matrix_lp2048x8192.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_digest") != source_digest() or t.get("m") != m or t.get("n") != n:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(lp, iters_gpu: int, sample_iters: int) -> dict:
    import oracle

    threads = oracle.num_threads()
    x, y, s = lp.x0, lp.y0, lp.s0
    t0 = time.perf_counter()
    for _ in range(sample_iters):
        it = oracle.iterate(lp.A, lp.b, lp.c, x, y, s, WORK["alpha"])
        x, y, s = it.x, it.y, it.s
    dt = (time.perf_counter() - t0) / sample_iters
    return {
        "value": 1.0 / (dt * max(iters_gpu, 1)),
        "unit": "LP solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{sample_iters} oracle iterations from the start point of the same LP, "
                   f"{dt:.2f} s each, scaled by the GPU's {iters_gpu} iterations per solve"),
    }


def batch_variant(lpgen, solver, capi, torch, sample: int = 32) -> dict:
    """512 ragged LPs (seeds 0..511) solved together vs. the single-LP FP64
    solver applied LP by LP to the first `sample` of them."""
    import numpy as np

    lps = lpgen.gen_batch(512, first_seed=0)
    warm = solver.Batch(lps, alpha=0.95)
    warm.solve(1e-8, 200)
    warm.close()
    bt = solver.Batch(lps, alpha=0.95)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = bt.solve(1e-8, 200)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    names = [capi.status_string(int(v)) for v in res["status"]]
    launch = {"batch_tile": int(bt.opts.batch_tile) or 64,
              "batch_graph_iters": int(bt.opts.batch_graph_iters) or 4,
              "source": "autotune cache" if solver.tuned_batch_launch(bt.m, bt.n)
              else "library default"}
    bt.close()
    # the same batch with the FP32 factor and FP64 refinement per LP
    wm = solver.Batch(lps, alpha=0.95, precision="mixed")
    wm.solve(1e-8, 200)
    wm.close()
    bm = solver.Batch(lps, alpha=0.95, precision="mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    resm = bm.solve(1e-8, 200)
    torch.cuda.synchronize()
    tm = time.perf_counter() - t0
    bm.close()
    # untimed: which factor each step used (lp_batch_iterate reports it)
    bi = solver.Batch(lps, alpha=0.95, precision="mixed")
    n32 = n64 = 0
    for _ in range(200):
        st_i, info = bi.iterate(1e-8)
        for e in info:
            if e["k"] >= 0:
                n32 += e["precision_used"] == capi.LP_PREC_MIXED
                n64 += e["precision_used"] != capi.LP_PREC_MIXED
        if not np.any(st_i == capi.LP_OK):
            break
    bi.close()
    mixed = {"lps_per_s": len(lps) / tm, "ms": tm * 1e3,
             "vs_fp64_batched": (len(lps) / tm) / (len(lps) / tb),
             "n_converged": int(resm["n_converged"]),
             "steps_with_fp32_factor": int(n32), "steps_with_fp64_factor": int(n64),
             "note": "FP32 normal matrix and factor, up to 5 FP64 corrections per step, FP64 "
                     "fallback per LP; FP64 below gap 1e-6"}
    dev = torch.device("cuda:0")
    hs = []
    for lp in lps[:sample]:
        T = [torch.from_numpy(np.ascontiguousarray(v)).to(dev)
             for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
        hs.append((solver.LP(*T, alpha=0.95), T))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h, _ in hs:
        h.solve(1e-8, 200)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    for h, _ in hs:
        h.close()
    return {
        "workload": "512 LPs, m ~ U{16..256}, n = round(r m), r ~ U(3,5), seeds 0..511, FP64, "
                    "alpha 0.95, to gap 1e-8",
        "batched_lps_per_s": len(lps) / tb,
        "batched_ms": tb * 1e3,
        "launch": launch,
        "mixed_precision": mixed,
        "fp64_lp_by_lp_lps_per_s": sample / ts,
        "lp_by_lp_sample": f"single-LP solver on LPs 0..{sample - 1}, one after another",
        "speedup_vs_lp_by_lp": (len(lps) / tb) / (sample / ts),
        "status_counts": {k: names.count(k) for k in sorted(set(names))},
        "iterations": {"max": int(np.max(res["iters"])), "mean": float(np.mean(res["iters"])),
                       "p90": float(np.percentile(res["iters"], 90))},
    }


def adjoint_variant(lpgen, solver, capi, torch, cpu: bool) -> dict:
    """64 LPs, m = 256, n = 1024 (seeds 0..63), exactly K = 30 steps at alpha
    0.9 with a tape, then the reverse sweep of w^T x_K: forward plus backward
    for the whole batch, timed after setup (a first run warms up).  With
    `cpu`, the oracle's forward K steps and reverse sweep for LP 0 beside it."""
    import numpy as np

    K, m, n, count = 30, 256, 1024, 64
    lps = [lpgen.gen_lp(m, n, i) for i in range(count)]
    wcat = torch.from_numpy(
        np.concatenate([lpgen.loss_weights(n, i) for i in range(count)])).to("cuda:0")

    def run():
        bt = solver.Batch(lps, alpha=0.9, tape_capacity=K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = bt.solve(0.0, K)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        bt.backward(wcat)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ok = all(capi.status_string(int(v)) == "LP_MAX_ITER" for v in res["status"])
        bt.close()
        return t1 - t0, t2 - t1, ok

    run()
    tf, tb, ok = run()
    out = {
        "workload": f"{count} LPs m={m} n={n} (seeds 0..{count - 1}), K={K} steps at alpha 0.9 "
                    "with a tape, then the reverse sweep of w^T x_K (w from stream 5), FP64",
        "lps_per_s": count / (tf + tb),
        "forward_ms": 1e3 * tf,
        "backward_ms": 1e3 * tb,
        "all_took_K_steps": ok,
    }
    if cpu:
        import oracle

        ns = 4
        t0 = time.perf_counter()
        for i in range(ns):
            lp = lps[i]
            r = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.9, 0.0, K, tape=True)
            oracle.backward(lp.A, lp.b, lp.c, 0.9, K, r.tape, lpgen.loss_weights(n, i))
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": ns / dt, "unit": "LPs/s (forward K steps + reverse sweep)",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"LPs 0..{ns - 1} of the {count}: oracle forward {K} steps with tape and "
                      f"reverse sweep, {dt:.2f} s"}
    return out


def mixed_variant(lpgen, solver, capi, torch) -> dict:
    """m=8192, n=32768 (seed 0): one FP64 solve and one mixed-precision solve
    from the same start to gap 1e-8, each timed whole (inputs resident, handle
    set up, one warm-up iteration on a separate handle first), with per-phase
    device times and the FP32 normal-matrix kernel's time on the iterations
    that kept the FP32 factor."""
    import numpy as np

    m, n = 8192, 32768
    dev = torch.device("cuda:0")
    lp = lpgen.gen_lp(m, n, 0)
    T = [torch.from_numpy(v).to(dev) for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
    del lp
    torch.cuda.synchronize()
    out = {"workload": "single LP m=8192 n=32768, Gaussian A (seed 0), alpha 0.95, to gap 1e-8: "
                       "mixed precision (FP32 normal matrix and factor, FP64 refinement and "
                       "fallback) vs plain FP64"}
    for prec in ("fp64", "mixed"):
        w = solver.LP(*T, alpha=0.95, precision=prec)
        w.iterate()
        w.close()
        h = solver.LP(*T, alpha=0.95, precision=prec, profile=True)
        torch.cuda.synchronize()
        fp32_kernel_ms, fp32_iters, prev = 0.0, 0, h.timings()
        t0 = time.perf_counter()
        # the loop of lp_solve, driven from here to attribute the FP32 kernel
        # time: stop once x^T s < 1e-8 after a step (the start gap is large)
        iters, st = 0, capi.LP_OK
        while True:
            info = h.iterate()
            iters += 1
            cur = h.timings()
            if info["precision_used"] == capi.LP_PREC_MIXED:
                fp32_kernel_ms += cur["normal_kernel_ms"] - prev["normal_kernel_ms"]
                fp32_iters += 1
            prev = cur
            if info["status"] != capi.LP_OK:
                st = info["status"]
                break
            if info["gap_after"] < 1e-8:
                st = capi.LP_CONVERGED
                break
            if iters >= 300:
                st = capi.LP_MAX_ITER
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = h.solve(1e-8, 0)  # objectives of the final iterate (no step taken)
        tim = h.timings()
        k = max(tim["iterations"], 1)
        out[prec] = {
            "status": capi.status_string(st), "iterations": iters, "seconds": dt,
            "dual_obj": res["dual_obj"],
            "ms_per_iteration": tim["iter_ms"] / k,
            "normal_matrix_ms_per_iteration": tim["normal_ms"] / k,
            "cholesky_ms_per_iteration": tim["potrf_ms"] / k,
            "triangular_solves_ms_per_iteration": tim["trsv_ms"] / k,
            "other_ms_per_iteration": tim["other_ms"] / k,
        }
        if prec == "mixed":
            out[prec]["fp32_iterations"] = fp32_iters
            out[prec]["fp32_normal_kernel_ms"] = fp32_kernel_ms / max(fp32_iters, 1)
        else:
            out[prec]["normal_kernel_ms"] = tim["normal_kernel_ms"] / max(tim["normal_launches"], 1)
        h.close()
    out["speedup_mixed_vs_fp64"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    out["dual_obj_rel_diff"] = abs(out["mixed"]["dual_obj"] - out["fp64"]["dual_obj"]) / max(
        1.0, abs(out["fp64"]["dual_obj"]))
    f64, mx = out["fp64"], out["mixed"]
    rl = []
    a = syrk_flops(m, n) / (f64["normal_kernel_ms"] * 1e-3) / 1e12
    rl.append({"kernel": "k_syrk_sk FP64 normal matrix, m=8192 n=32768", "bound": "mfma",
               "achieved": a, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
               "frac": a / PEAK_FP64_MFMA_TFLOPS})
    a = potrf_flops(m) / (f64["cholesky_ms_per_iteration"] * 1e-3) / 1e12
    rl.append({"kernel": "FP64 Cholesky (all launches of one factorization), m=8192",
               "bound": "mfma", "achieved": a, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
               "frac": a / PEAK_FP64_MFMA_TFLOPS})
    if mx.get("fp32_iterations"):
        a = syrk_flops(m, n) / (mx["fp32_normal_kernel_ms"] * 1e-3) / 1e12
        rl.append({"kernel": "FP32 normal matrix (mixed precision), m=8192 n=32768",
                   "bound": "mfma", "achieved": a, "peak": PEAK_FP32_MFMA_TFLOPS,
                   "unit": "TFLOP/s", "frac": a / PEAK_FP32_MFMA_TFLOPS})
    out["rooflines"] = rl
    del T
    torch.cuda.empty_cache()
    return out


def pc_variant(lpgen, solver, capi, torch, T, m, n, affine_solves_per_s, steps=5) -> dict:
    """The same instance as the main line, solved by the predictor-corrector
    variant (one factorization and two solves per iteration) to the same gap:
    LP solves/s beside the Section 3 algorithm's."""
    handles = [solver.LP(*T, alpha=0.95, method="pc", profile=True) for _ in range(steps + 1)]
    handles[0].solve(1e-8, 100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [h.solve(1e-8, 100) for h in handles[1:]]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tims = [h.timings() for h in handles[1:]]
    tot = {k: sum(t[k] for t in tims) for k in tims[0]}
    out = {
        "workload": f"single LP m={m} n={n} (the main line's instance), Mehrotra "
                    "predictor-corrector, eta 0.95, to gap 1e-8, FP64",
        "lp_solves_per_s": steps / wall,
        "ms_per_solve": wall * 1e3 / steps,
        "iterations_per_solve": res[0]["iters"],
        "statuses": sorted({capi.status_string(r["status"]) for r in res}),
        "ms_per_iteration": tot["iter_ms"] / max(tot["iterations"], 1),
        "dual_obj": res[0]["dual_obj"],
        "speedup_vs_affine_scaling": (steps / wall) / affine_solves_per_s,
    }
    for h in handles:
        h.close()
    return out


def woodbury_variant(lpgen, solver, capi, torch, steps=20) -> dict:
    """m=64, n=256 (seed 0): the paper's Woodbury / Egidi-Maponi direction
    solver against the normal-matrix + Cholesky path, whole solves to gap
    1e-8 with inputs resident, and the recurrence kernel's rate (about
    2 m n^2 flops per iteration, in one compute unit) against that compute
    unit's FP64 vector peak."""
    import numpy as np

    m, n = 64, 256
    lp = lpgen.gen_lp(m, n, 0)
    dev = torch.device("cuda:0")
    T = [torch.from_numpy(np.ascontiguousarray(v)).to(dev)
         for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
    out = {"workload": f"single LP m={m} n={n} (seed 0), alpha 0.95, to gap 1e-8, FP64"}
    for name in ("woodbury", "cholesky"):
        hs = [solver.LP(*T, alpha=0.95, solver=name, profile=True) for _ in range(steps + 1)]
        hs[0].solve(1e-8, 200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [h.solve(1e-8, 200) for h in hs[1:]]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tims = [h.timings() for h in hs[1:]]
        tot = {k: sum(t[k] for t in tims) for k in tims[0]}
        it = max(tot["iterations"], 1)
        out[name] = {"lp_solves_per_s": steps / wall, "iterations_per_solve": res[0]["iters"],
                     "statuses": sorted({capi.status_string(r["status"]) for r in res}),
                     "dual_obj": res[0]["dual_obj"], "ms_per_iteration": tot["iter_ms"] / it,
                     "direction_solve_ms_per_iteration":
                         (tot["normal_ms"] + tot["potrf_ms"] + tot["trsv_ms"]) / it}
        if name == "woodbury":
            flops = 2.0 * m * n * n
            ms = tot["potrf_ms"] / it  # x0 solves plus the recurrence kernel
            a = flops / (ms * 1e-3) / 1e9
            peak_cu = PEAK_FP64_MFMA_TFLOPS * 1e3 / 256  # one CU's share, GFLOP/s
            out[name]["recurrence_roofline"] = {
                "kernel": "k_woodbury (n rank-one terms in one workgroup, Y in LDS)",
                "bound": "lds/latency (one compute unit)", "achieved": a, "peak": peak_cu,
                "unit": "GFLOP/s", "frac": a / peak_cu, "algorithmic_flops_per_launch": flops,
                "avg_ms": ms}
        for h in hs:
            h.close()
    out["woodbury_vs_cholesky"] = (out["woodbury"]["lp_solves_per_s"] /
                                   out["cholesky"]["lp_solves_per_s"])
    return out


def sparse_variant(lpgen, solver, capi, torch, steps=5) -> dict:
    """m=2048, n=8192 with 1% of A's entries nonzero (seed 0): whole solves
    to gap 1e-8 through lp_setup_csr against the dense path on the same
    matrix, and the sparse normal-matrix kernel's rate.  Its algorithmic
    HBM bytes per launch: the lower triangle of M written once (8 m (m+1)/2)
    plus the CSR and CSC entries read once (12 bytes each); its multiply-adds
    are sum over columns c_k (c_k + 1) / 2 (c_k entries in column k)."""
    import numpy as np

    m, n, density = 2048, 8192, 0.01
    lp = lpgen.gen_sparse_lp(m, n, density, 0)
    dev = torch.device("cuda:0")
    dense = [torch.from_numpy(np.ascontiguousarray(v)).to(dev)
             for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
    csr = (torch.from_numpy(lp.row_ptr).to(dev), torch.from_numpy(lp.col_idx).to(dev),
           torch.from_numpy(lp.vals).to(dev))
    out = {"workload": f"single LP m={m} n={n}, density {density} (nnz {lp.nnz}, seed 0), "
                       "alpha 0.95, to gap 1e-8, FP64"}
    for name in ("csr", "dense"):
        def make():
            if name == "csr":
                return solver.CsrLP(*csr, (m, n), *dense[1:], alpha=0.95, profile=True)
            return solver.LP(*dense, alpha=0.95, profile=True)
        hs = [make() for _ in range(steps + 1)]
        hs[0].solve(1e-8, 200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [h.solve(1e-8, 200) for h in hs[1:]]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tims = [h.timings() for h in hs[1:]]
        tot = {k: sum(t[k] for t in tims) for k in tims[0]}
        it = max(tot["iterations"], 1)
        out[name] = {"lp_solves_per_s": steps / wall, "iterations_per_solve": res[0]["iters"],
                     "statuses": sorted({capi.status_string(r["status"]) for r in res}),
                     "dual_obj": res[0]["dual_obj"], "ms_per_iteration": tot["iter_ms"] / it,
                     "normal_matrix_ms": tot["normal_kernel_ms"] / it,
                     "cholesky_ms": tot["potrf_ms"] / it, "trsv_ms": tot["trsv_ms"] / it,
                     "other_ms": tot["other_ms"] / it}
        if name == "csr":
            cnt = np.bincount(lp.col_idx, minlength=n).astype(np.float64)
            fmas = float(np.sum(cnt * (cnt + 1) / 2))
            nbytes = 8.0 * m * (m + 1) / 2 + 2 * 12.0 * lp.nnz
            ms = tot["normal_kernel_ms"] / it
            gbs = nbytes / (ms * 1e-3) / 1e9
            out[name]["normal_matrix_roofline"] = {
                "kernel": "k_sp_syrk (row i of M per workgroup, LDS accumulator)",
                "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": gbs / PEAK_HBM_GBS, "algorithmic_bytes_per_launch": nbytes,
                "multiply_adds_per_launch": fmas, "avg_ms": ms}
        for h in hs:
            h.close()
    out["csr_vs_dense"] = out["csr"]["lp_solves_per_s"] / out["dense"]["lp_solves_per_s"]
    return out


def mixed_compare():
    """m=8192, n=32768: one mixed-precision solve and one FP64 solve from the
    same start, with the per-iteration precision and refinement counts."""
    import numpy as np
    import torch

    from paper_1502_03543_amd import capi, lpgen, solver

    capi.load()
    dev = torch.device("cuda:0")
    lp = lpgen.gen_lp(8192, 32768, 0)
    T = [torch.from_numpy(v).to(dev) for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
    del lp
    out = {"workload": "single LP m=8192 n=32768, Gaussian A, alpha 0.95, to gap 1e-8"}
    runs = (("mixed", "mixed", {}), ("mixed_refine12", "mixed", {"refine_max": 12}),
            ("fp64", "fp64", {}))
    for name, prec, extra in runs:
        h = solver.LP(*T, alpha=0.95, precision=prec, profile=True, **extra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = h.solve(1e-8, 300, want_log=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tim = h.timings()
        log = r.get("log") or []
        out[name] = {
            "status": capi.status_string(r["status"]), "iterations": r["iters"] + 1,
            "seconds": dt, "dual_obj": r["dual_obj"],
            "fp32_iterations": sum(1 for e in log if e["precision_used"] == capi.LP_PREC_MIXED),
            "refine_steps": [e["refine_steps"] for e in log],
            "ms_per_iteration": tim["iter_ms"] / max(tim["iterations"], 1),
            "normal_ms_per_iteration": tim["normal_ms"] / max(tim["iterations"], 1),
            "cholesky_ms_per_iteration": tim["potrf_ms"] / max(tim["iterations"], 1),
        }
        h.close()
        print(json.dumps({name: out[name]}), flush=True)
    out["speedup_mixed_vs_fp64"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    out["speedup_mixed_refine12_vs_fp64"] = out["fp64"]["seconds"] / out["mixed_refine12"]["seconds"]
    out["dual_obj_rel_diff"] = abs(out["mixed"]["dual_obj"] - out["fp64"]["dual_obj"]) / max(
        1.0, abs(out["fp64"]["dual_obj"]))
    print(json.dumps(out))


def copy_probe():
    import torch

    n = 32 * 1024 * 1024  # 256 MiB of float64
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 8 * n, "copy_probe_bytes_written": 8 * n,
                      "launches": 5}))


def main():
    global WORK
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lp2048x8192", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=3)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--mixed-compare", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--variant", choices=("batched", "sparse", "adjoint", "woodbury"),
                    help="run only this variant and print its JSON (for profiling)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (the solver runs on a single "
              "MI355X); multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.mixed_compare:
        mixed_compare()
        return
    if args.variant:
        import torch

        from paper_1502_03543_amd import capi, lpgen, solver

        capi.load()
        run = {"batched": lambda: batch_variant(lpgen, solver, capi, torch),
               "sparse": lambda: sparse_variant(lpgen, solver, capi, torch),
               "adjoint": lambda: adjoint_variant(lpgen, solver, capi, torch, False),
               "woodbury": lambda: woodbury_variant(lpgen, solver, capi, torch)}[args.variant]
        print(json.dumps({"variant": args.variant, **run()}))
        return

    import numpy as np
    import torch

    from paper_1502_03543_amd import capi, lpgen, solver

    WORK = WORKLOADS[args.workload]
    m, n = WORK["m"], WORK["n"]
    capi.load()
    dev = torch.device("cuda:0")
    lp = lpgen.gen_lp(m, n, WORK["seed"])
    T = [torch.from_numpy(v).to(dev) for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0)]
    torch.cuda.synchronize()

    # handles are set up before the timed region (setup time reported apart).
    # The timed solves record two HIP events per iteration, around the
    # normal-matrix kernel (the roofline's launch time); the per-phase split
    # comes from two more solves, after the timed region, with every phase's
    # events (those cost about 2% of a solve, so they stay out of the timing)
    t0 = time.perf_counter()
    handles = [solver.LP(*T, alpha=WORK["alpha"], profile="kernel")
               for _ in range(args.warmup + args.steps)]
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3 / len(handles)
    phase_handles = [solver.LP(*T, alpha=WORK["alpha"], profile=True) for _ in range(2)]
    torch.cuda.synchronize()

    results = []
    for h in handles[: args.warmup]:
        results.append(h.solve(WORK["tol"], 500))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed = []
    for h in handles[args.warmup:]:
        timed.append(h.solve(WORK["tol"], 500))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    statuses = sorted({capi.status_string(r["status"]) for r in timed})
    iters = [r["iters"] for r in timed]
    if statuses != ["LP_CONVERGED"] or len(set(iters)) != 1:
        print(json.dumps({"error": "solves did not all converge identically",
                          "statuses": statuses, "iters": iters}), file=sys.stderr)
        sys.exit(1)
    K = iters[0]

    ktims = [h.timings() for h in handles[args.warmup:]]
    launches = sum(t["normal_launches"] for t in ktims)
    kernel_ms = sum(t["normal_kernel_ms"] for t in ktims) / launches
    for h in phase_handles:
        r = h.solve(WORK["tol"], 500)
        if capi.status_string(r["status"]) != "LP_CONVERGED" or r["iters"] != K:
            print(json.dumps({"error": "phase-timing solve differs", "iters": r["iters"]}),
                  file=sys.stderr)
            sys.exit(1)
    torch.cuda.synchronize()
    tims = [h.timings() for h in phase_handles]
    tot = {k: sum(t[k] for t in tims) for k in tims[0]}
    achieved_tflops = syrk_flops(m, n) / (kernel_ms * 1e-3) / 1e12
    gflops_s4s5 = (tot["iterations"] * (syrk_flops(m, n) + potrf_flops(m))
                   / ((tot["normal_ms"] + tot["potrf_ms"]) * 1e-3) / 1e9)
    traffic = read_traffic(m, n)
    o = handles[0].opts
    if o.syrk_tile == 0 and o.syrk_splits == 0 and m >= 512 and n >= 1024:
        kname = ("k_syrk_sk (normal matrix A D A^T, stream-K: 128x128 lower tiles, one equal "
                 "share of tile-stages per compute unit, v_mfma_f64_16x16x4f64)")
    else:
        kname = (f"k_syrk_f64 (normal matrix A D A^T, lower {o.syrk_tile or 'library-chosen'} "
                 f"tiles, split-K {o.syrk_splits or 'library-chosen'})")

    out = {
        "metric": "LP solves/s (ADA^T + Cholesky GFLOP/s reported alongside)",
        "value": args.steps / wall,
        "unit": "LP solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian interior-feasible LP generator)",
        "config": {"workload": WORK["desc"], "m": m, "n": n, "seed": WORK["seed"],
                   "alpha": WORK["alpha"], "gap_tol": WORK["tol"], "iterations_per_solve": K,
                   "parallelism": "single GPU"},
        "gflops_normal_plus_cholesky": gflops_s4s5,
        "phase_ms_per_iteration": {
            "normal_matrix_kernel": kernel_ms,
            "normal_matrix_total": tot["normal_ms"] / tot["iterations"],
            "cholesky": tot["potrf_ms"] / tot["iterations"],
            "triangular_solves": tot["trsv_ms"] / tot["iterations"],
            "gemv_direction_step": tot["other_ms"] / tot["iterations"],
            "iteration": tot["iter_ms"] / tot["iterations"],
        },
        "setup_ms": setup_ms,
        "roofline": {
            "kernel": kname,
            "bound": "mfma",
            "achieved": achieved_tflops,
            "peak": PEAK_FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP64_MFMA_TFLOPS,
            "traffic": traffic,
            "algorithmic_flops_per_launch": syrk_flops(m, n),
            "avg_launch_ms": kernel_ms,
        },
    }
    for h in handles:
        h.close()
    a = potrf_flops(m) / (tot["potrf_ms"] / tot["iterations"] * 1e-3) / 1e12
    out["rooflines_other"] = [{
        "kernel": f"FP64 Cholesky (all launches of one factorization), m={m}", "bound": "mfma",
        "achieved": a, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
        "frac": a / PEAK_FP64_MFMA_TFLOPS,
        "algorithmic_flops_per_factorization": potrf_flops(m),
        "avg_ms": tot["potrf_ms"] / tot["iterations"]}]
    if not args.no_variants:
        out["variants"] = {
            "predictor_corrector": pc_variant(lpgen, solver, capi, torch, T, m, n,
                                              out["value"]),
            "woodbury": woodbury_variant(lpgen, solver, capi, torch),
            "batched": batch_variant(lpgen, solver, capi, torch),
            "adjoint": adjoint_variant(lpgen, solver, capi, torch, not args.no_cpu_baseline),
            "mixed": mixed_variant(lpgen, solver, capi, torch),
            "sparse": sparse_variant(lpgen, solver, capi, torch),
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(lp, K, args.cpu_sample_iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
