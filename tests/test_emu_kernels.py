"""Kernel logic on the CPU: the HIP sources of the Cholesky (panel routine,
trailing update, forward solve fused as an extra row) and of the batched
solver (forward and reverse sweeps) run under the host emulation of
tests/emu (workgroups as fibers, wavefront lock-step, AddressSanitizer), and
and the sparse-A kernels (CSR check, transpose, products, normal matrix)
are checked against a long-double reference and against the oracle.

These tests run without a GPU; they check indexing, synchronisation and the
algorithm, not the hardware's rounding (the emulated matrix-core and
reciprocal-square-root instructions are exact-rounded host operations)."""
import importlib.util
import json
import os
import struct
import subprocess

import numpy as np
import pytest

import oracle
from paper_1502_03543_amd import lpgen

_spec = importlib.util.spec_from_file_location(
    "build_emu", os.path.join(os.path.dirname(os.path.abspath(__file__)), "emu", "build_emu.py"))
build_emu = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(build_emu)

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0")


@pytest.fixture(scope="module")
def emu():
    if build_emu.compiler() is None:
        pytest.skip("no clang++ for the kernel emulation")
    return build_emu.build()


def _run(exe, *args, timeout=600, interleave=1):
    env = dict(ENV, EMU_INTERLEAVE=str(interleave))
    p = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=timeout,
                       env=env)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    return p.stdout


@pytest.mark.parametrize("m,group", [(40, 0), (64, 0), (100, 0), (150, 0), (300, 0), (700, 0),
                                     (1100, 0), (300, 128), (700, 256), (1100, 256)])
def test_emulated_cholesky_with_fused_forward_solve(emu, m, group):
    """group > 0: the grouped schedule of large matrices (panels by four; at a
    group's end its update of the next panel's columns, of the rest of the
    next group beside that group's first panel on 64-edge tiles, and of the
    columns beyond the next group as a launch of its own) at a small m: with
    300 the second group is the last (no update beyond it); 700 and 1100 end
    in a ragged group."""
    r = json.loads(_run(emu, "chol", m, group).strip().splitlines()[-1])
    assert r["fail"] == -1
    assert r["factor_rel_err"] <= 1e-13, r
    assert r["solve_rel_err"] <= 1e-13, r
    assert r["min_pivot_rel_err"] <= 1e-13, r


@pytest.mark.parametrize("m,n,tile,splits", [(150, 301, 128, 3), (200, 333, 64, 4),
                                             (130, 257, 128, 1), (70, 190, 64, 2),
                                             (150, 302, 0, 0), (260, 98, 0, 0),
                                             (100, 40, 0, 0)])
def test_emulated_normal_matrix(emu, m, n, tile, splits):
    r = json.loads(_run(emu, "syrk", m, n, tile, splits).strip().splitlines()[-1])
    assert r["rel_err"] <= 1e-14, r


@pytest.mark.parametrize("m", [1, 40, 64, 100, 200, 300])
def test_emulated_triangular_solves(emu, m):
    r = json.loads(_run(emu, "trsv", m).strip().splitlines()[-1])
    assert r["err_flag"] == 0, r
    assert r["fwd_rel_err"] <= 1e-13, r
    assert r["bwd_rel_err"] <= 1e-13, r


@pytest.mark.parametrize("m,n,pattern", [(3, 9, 1), (300, 700, 0), (2200, 2600, 0),
                                         (100, 300, 1)])
def test_emulated_sparse_kernels(emu, m, n, pattern):
    """CSR check, CSC build, both products and the sparse normal matrix.
    Pattern 0 reaches every branch of the normal-matrix kernel: a row of 300
    entries (five 64-entry chunks), runs longer than a wavefront (the dense
    column), empty rows and columns; pattern 1 takes the 64-lane products."""
    r = json.loads(_run(emu, "sparse", m, n, pattern).strip().splitlines()[-1])
    assert r["flags"] == 0 and r["csc_bad"] == 0 and r["upper_touched"] == 0, r
    assert r["gemv_n_rel_err"] <= 1e-15 and r["gemv_t_rel_err"] <= 1e-15, r
    assert r["syrk_rel_err"] <= 1e-14, r
    assert (r["f_unsorted"], r["f_range"], r["f_nan"], r["f_count"], r["f_order"]) == \
        (1, 1, 2, 1, 1), r


def _write(path, lps):
    with open(path, "wb") as f:
        f.write(struct.pack("i", len(lps)))
        for lp in lps:
            m, n = lp.A.shape
            f.write(struct.pack("qq", m, n))
            for v in (lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0):
                f.write(np.ascontiguousarray(v, dtype=np.float64).tobytes())


def _lps():
    lps = [lpgen.gen_lp(40, 150, 3), lpgen.gen_lp(70, 260, 4), lpgen.gen_lp(33, 101, 5)]
    bad = lpgen.gen_lp(30, 90, 6)
    bad.A = bad.A.copy()
    bad.A[3] = 0.0                      # zero row: exact zero pivot in this LP only
    bad.b = bad.A @ bad.x0
    return lps + [bad]


@pytest.mark.parametrize("tile", [0, 32, 128])
def test_emulated_batch_matches_oracle(emu, tmp_path, tile):
    lps = _lps()
    if tile in (0, 128):
        lps.append(lpgen.gen_lp(150, 331, 7))   # 64-edge tiles / two 128-row tiles, ragged
    _write(tmp_path / "in.bin", lps)
    _run(emu, "batch", tmp_path / "in.bin", tmp_path / "out.bin", 200, 0, tile)
    raw = (tmp_path / "out.bin").read_bytes()
    k = len(lps)
    st = np.frombuffer(raw[:4 * k], np.int32)
    it = np.frombuffer(raw[4 * k:8 * k], np.int32)
    sn = sum(lp.A.shape[1] for lp in lps)
    y = np.frombuffer(raw[8 * k:], np.float64)[sn:]
    names = {1: "CONVERGED", 2: "OPTIMAL_PSI1", -4: "ERR_BREAKDOWN"}
    om = 0
    for i, lp in enumerate(lps):
        m = lp.A.shape[0]
        ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
        assert names.get(int(st[i])) == ro.status_name, (i, st[i], ro.status_name)
        assert it[i] == ro.iters
        if ro.status == oracle.CONVERGED:
            byo = lp.b @ ro.y
            assert abs(lp.b @ y[om:om + m] - byo) <= 1e-9 * max(1.0, abs(byo))
        om += m


def test_emulated_batch_mixed_precision(emu, tmp_path):
    """The batch with the FP32 factor and FP64 refinement per LP: statuses,
    iteration counts and b^T y as the FP64 oracle; the LP with a zero row
    fails its FP32 pivot, falls back to FP64 and breaks down there."""
    lps = _lps()
    _write(tmp_path / "in.bin", lps)
    _run(emu, "batch", tmp_path / "in.bin", tmp_path / "out.bin", 200, 0, 0, 1)
    raw = (tmp_path / "out.bin").read_bytes()
    k = len(lps)
    st = np.frombuffer(raw[:4 * k], np.int32)
    it = np.frombuffer(raw[4 * k:8 * k], np.int32)
    sn = sum(lp.A.shape[1] for lp in lps)
    y = np.frombuffer(raw[8 * k:], np.float64)[sn:]
    names = {1: "CONVERGED", 2: "OPTIMAL_PSI1", -4: "ERR_BREAKDOWN"}
    om = 0
    for i, lp in enumerate(lps):
        m = lp.A.shape[0]
        ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
        assert names.get(int(st[i])) == ro.status_name, (i, st[i], ro.status_name)
        assert it[i] == ro.iters
        if ro.status == oracle.CONVERGED:
            byo = lp.b @ ro.y
            assert abs(lp.b @ y[om:om + m] - byo) <= 1e-9 * max(1.0, abs(byo))
        om += m


@pytest.mark.parametrize("mixed", [0, 1])
def test_emulated_batch_compaction(emu, tmp_path, mixed):
    """Twelve LPs of very different sizes: the batch is compacted (running
    LPs moved to the first slots, the launches re-shaped for them) as the
    small ones finish, in FP64 and with the per-LP FP32 factor (whose flags
    move with their LPs); every LP still matches the oracle's solve."""
    lps = [lpgen.gen_lp(m, n, 40 + i) for i, (m, n) in enumerate(
        [(6, 20), (90, 300), (8, 30), (12, 40), (70, 260), (5, 17), (10, 33), (16, 60),
         (9, 28), (130, 420), (7, 25), (11, 35)])]
    _write(tmp_path / "in.bin", lps)
    _run(emu, "batch", tmp_path / "in.bin", tmp_path / "out.bin", 200, 0, 0, mixed)
    raw = (tmp_path / "out.bin").read_bytes()
    k = len(lps)
    st = np.frombuffer(raw[:4 * k], np.int32)
    it = np.frombuffer(raw[4 * k:8 * k], np.int32)
    sn = sum(lp.A.shape[1] for lp in lps)
    y = np.frombuffer(raw[8 * k:], np.float64)[sn:]
    om = 0
    for i, lp in enumerate(lps):
        m = lp.A.shape[0]
        ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
        assert ro.status == oracle.CONVERGED and st[i] == 1, (i, st[i], ro.status_name)
        assert it[i] == ro.iters, (i, it[i], ro.iters)
        byo = lp.b @ ro.y
        assert abs(lp.b @ y[om:om + m] - byo) <= 1e-9 * max(1.0, abs(byo))
        om += m
    assert len(set(it.tolist())) > 1  # the LPs finish at different iterations


def test_emulated_batch_reverse_matches_oracle(emu, tmp_path):
    K = 3
    lps = _lps()[:3]
    _write(tmp_path / "in.bin", lps)
    _run(emu, "batch", tmp_path / "in.bin", tmp_path / "out.bin", K, K)
    raw = np.frombuffer((tmp_path / "out.bin").read_bytes()[8 * len(lps):], np.float64)
    ms = [lp.A.shape[0] for lp in lps]
    ns = [lp.A.shape[1] for lp in lps]
    sm, sn, sa = sum(ms), sum(ns), sum(a * b for a, b in zip(ms, ns))
    g = raw[2 * sn + sm:]
    Ab, bb, cb = g[:sa], g[sa:sa + sm], g[sa + sm:sa + sm + sn]
    rows = g[sa + sm + sn:].reshape(K, 2 * sn + sm)
    ao = vm = vn = 0
    for lp, m, n in zip(lps, ms, ns):
        tape = np.stack([np.concatenate([r[vn:vn + n], r[sn + vm:sn + vm + m],
                                         r[sn + sm + vn:sn + sm + vn + n]]) for r in rows])
        xb = np.sin(0.37 * np.arange(vn, vn + n) + 0.1)
        st, go = oracle.backward(lp.A, lp.b, lp.c, 0.95, K, tape, xb)
        assert st == oracle.CONTINUE
        for got, ref in ((Ab[ao:ao + m * n].reshape(m, n), go["Abar"]),
                         (bb[vm:vm + m], go["bbar"]), (cb[vn:vn + n], go["cbar"])):
            assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
        ao += m * n
        vm += m
        vn += n


@pytest.mark.parametrize("case", ["trsv", "chol", "syrk", "sparse", "batch"])
def test_emulated_kernels_interleaved(emu, tmp_path, case):
    """Workgroups run four or eight at a time on their own OS threads, so
    they interleave at arbitrary points: the ticketed triangular solves
    poll blocks that are still running, the fused Cholesky step's panel and
    update workgroups overlap, the batched solver's workgroups take LPs
    concurrently.  Results as in the sequential runs; any barrier reached
    unevenly aborts the run."""
    if case == "trsv":
        r = json.loads(_run(emu, "trsv", 700, interleave=8).strip().splitlines()[-1])
        assert r["err_flag"] == 0 and r["fwd_rel_err"] <= 1e-13 and r["bwd_rel_err"] <= 1e-13, r
    elif case == "chol":
        r = json.loads(_run(emu, "chol", 300, interleave=4).strip().splitlines()[-1])
        assert r["fail"] == -1 and r["factor_rel_err"] <= 1e-13 and r["solve_rel_err"] <= 1e-13, r
    elif case == "syrk":
        r = json.loads(_run(emu, "syrk", 150, 302, 0, 0, interleave=4).strip().splitlines()[-1])
        assert r["rel_err"] <= 1e-14, r
    elif case == "sparse":
        r = json.loads(_run(emu, "sparse", 2200, 2600, 0, interleave=8).strip().splitlines()[-1])
        assert r["flags"] == 0 and r["csc_bad"] == 0 and r["syrk_rel_err"] <= 1e-14, r
    else:
        lps = _lps()
        _write(tmp_path / "in.bin", lps)
        _run(emu, "batch", tmp_path / "in.bin", tmp_path / "out.bin", 200, 0, 0, 1, interleave=4)
        raw = (tmp_path / "out.bin").read_bytes()
        k = len(lps)
        st = np.frombuffer(raw[:4 * k], np.int32)
        it = np.frombuffer(raw[4 * k:8 * k], np.int32)
        for i, lp in enumerate(lps):
            ro = oracle.solve(lp.A, lp.b, lp.c, lp.x0, lp.y0, lp.s0, 0.95, 1e-8, 200)
            assert it[i] == ro.iters and (st[i] == 1) == (ro.status == oracle.CONVERGED), i
