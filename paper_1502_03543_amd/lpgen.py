"""Seeded synthetic LP instances (inputs only; none of the method's arithmetic).

Every instance is interior-feasible by construction, as the Section 3
algorithm requires of its start point: with A ~ N(0,1) (m x n, row-major),
x0, s0 ~ U(0.5, 1.5) and y0 ~ N(0,1), setting b = A x0 and c = A^T y0 + s0
makes x0 primal-feasible and (y0, s0) dual-feasible, so the LP is bounded
and x0, s0 > 0 is a valid interior start.

Random streams: numpy's Philox counter-based generator seeded with
SeedSequence([seed, stream]); stream 0 = A, 1 = x0, 2 = s0, 3 = y0,
4 = batch shape, 5 = loss weights w, 6 = the sparsity pattern of a sparse A.  b and c are computed once here, in
float64, and the same bytes feed both the GPU path and the oracle.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

STREAM_A, STREAM_X0, STREAM_S0, STREAM_Y0, STREAM_SHAPE, STREAM_W, STREAM_PATTERN = range(7)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), stream])))


@dataclass
class LP:
    A: np.ndarray   # (m, n) float64, C-contiguous
    b: np.ndarray   # (m,)
    c: np.ndarray   # (n,)
    x0: np.ndarray  # (n,)
    y0: np.ndarray  # (m,)
    s0: np.ndarray  # (n,)
    seed: int

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


def gen_lp(m: int, n: int, seed: int = 0) -> LP:
    """Gaussian interior-feasible LP of shape (m, n)."""
    if not (1 <= m < n):
        raise ValueError(f"need 1 <= m < n, got m={m} n={n}")
    A = _rng(seed, STREAM_A).standard_normal((m, n))
    x0 = 0.5 + _rng(seed, STREAM_X0).random(n)
    s0 = 0.5 + _rng(seed, STREAM_S0).random(n)
    y0 = _rng(seed, STREAM_Y0).standard_normal(m)
    b = A @ x0
    c = A.T @ y0 + s0
    return LP(A=np.ascontiguousarray(A), b=b, c=c, x0=x0, y0=y0, s0=s0, seed=seed)


def batch_shape(seed: int, m_lo: int = 16, m_hi: int = 256, r_lo: float = 3.0,
                r_hi: float = 5.0) -> tuple[int, int]:
    """(m, n) of batch member ``seed``: m ~ U{m_lo..m_hi}, n = round(r m) with
    r ~ U(r_lo, r_hi), rounded half to even."""
    u = _rng(seed, STREAM_SHAPE).random(2)
    m = m_lo + int(np.floor(u[0] * (m_hi - m_lo + 1)))
    m = min(m, m_hi)
    r = r_lo + (r_hi - r_lo) * u[1]
    n = int(np.round(r * m))
    return m, n


def gen_batch(count: int, first_seed: int = 0, **shape_kw) -> list[LP]:
    """Ragged batch: member i has seed first_seed + i and its own shape."""
    out = []
    for i in range(count):
        sd = first_seed + i
        m, n = batch_shape(sd, **shape_kw)
        out.append(gen_lp(m, n, sd))
    return out


def loss_weights(n: int, seed: int) -> np.ndarray:
    """w ~ N(0,1) for the loss w^T x_K."""
    return _rng(seed, STREAM_W).standard_normal(n)


@dataclass
class SparseLP(LP):
    """An LP whose A is sparse: CSR arrays beside the dense A (the dense copy
    serves the oracle; the GPU path takes the CSR arrays)."""
    row_ptr: np.ndarray = None  # (m + 1,) int64
    col_idx: np.ndarray = None  # (nnz,) int32, sorted within each row
    vals: np.ndarray = None     # (nnz,) float64

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def gen_sparse_lp(m: int, n: int, density: float, seed: int = 0) -> SparseLP:
    """Sparse interior-feasible LP: every row has a nonzero in its own column
    of a random permutation (so A has full row rank with probability one)
    plus each other entry independently with probability ``density``; the
    nonzero values are N(0,1); x0, s0, y0, b and c as in gen_lp."""
    if not (1 <= m < n) or not (0.0 < density <= 1.0):
        raise ValueError(f"need 1 <= m < n and 0 < density <= 1, got {m} {n} {density}")
    pat = _rng(seed, STREAM_PATTERN)
    mask = pat.random((m, n)) < density
    perm = pat.permutation(n)[:m]
    mask[np.arange(m), perm] = True
    vals_all = _rng(seed, STREAM_A).standard_normal((m, n))
    A = np.where(mask, vals_all, 0.0)
    x0 = 0.5 + _rng(seed, STREAM_X0).random(n)
    s0 = 0.5 + _rng(seed, STREAM_S0).random(n)
    y0 = _rng(seed, STREAM_Y0).standard_normal(m)
    b = A @ x0
    c = A.T @ y0 + s0
    rows, cols = np.nonzero(mask)  # row-major order: sorted columns within rows
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return SparseLP(A=np.ascontiguousarray(A), b=b, c=c, x0=x0, y0=y0, s0=s0, seed=seed,
                    row_ptr=row_ptr, col_idx=cols.astype(np.int32),
                    vals=np.ascontiguousarray(A[rows, cols]))
