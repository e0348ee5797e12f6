"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random matrices; it holds none of the Gram-product
arithmetic, and both the oracle tests and the GPU tests/benchmark use it.

The paper evaluates on randomly generated dense matrices (Sec. 5.1) without
naming a distribution or a dataset, so nothing external is stood in for.  The
recipes below fix the distribution, the seed and the draw order; all draws
use ``numpy.random.default_rng(seed)`` (PCG64) in float64 and are then cast
with round-to-nearest-even.  Row-chunked generation from one Generator gives
the same stream as a single call, which keeps host memory bounded.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_CHUNK_ELEMS = 1 << 24


@dataclass(frozen=True)
class Workload:
    name: str
    dtype: str            # "f64" or "f32"
    rows: int
    cols: int
    seed: int
    kind: str             # "uniform", "scaled_normal", "normal", "batch"
    description: str


WORKLOADS = {
    "square_f64_1024": Workload(
        "square_f64_1024", "f64", 1024, 1024, 1, "uniform",
        "A 1024x1024, i.i.d. uniform[-1,1], FP64; leaf cutoff 256"),
    "square_f32_8192": Workload(
        "square_f32_8192", "f32", 8192, 8192, 2, "uniform",
        "A 8192x8192, i.i.d. uniform[-1,1], FP32"),
    "tall_scaled_f32_262144x4096": Workload(
        "tall_scaled_f32_262144x4096", "f32", 262144, 4096, 3, "scaled_normal",
        "A 262144x4096, N(0,1) with column j scaled by 10^u_j, u_j ~ U[-3,3], FP32"),
    "normal_f32_16384": Workload(
        "normal_f32_16384", "f32", 16384, 16384, 4, "normal",
        "A 16384x16384, i.i.d. N(0,1), FP32; 256 sampled columns"),
    # the square sizes of the paper's shared- vs distributed-memory table
    # (Sec. 5), for context beside its CPU times
    **{f"paper_square_f64_{k}": Workload(
        f"paper_square_f64_{k}", "f64", k, k, k // 1000, "uniform",
        f"A {k}x{k}, i.i.d. uniform[-1,1], FP64 (a square size of the paper's Sec. 5 table)")
       for k in (30000, 40000, 50000, 60000)},
    "batch_512_uneven_f32": Workload(
        "batch_512_uneven_f32", "f32", 0, 0, 5, "batch",
        "512 problems, m log-uniform in [256,8192], n log-uniform in [64,2048], "
        "uniform[-1,1], FP32"),
}


def _fill(rng, rows, cols, draw, out_dtype):
    out = np.empty((rows, cols), dtype=out_dtype)
    step = max(1, _CHUNK_ELEMS // max(cols, 1))
    for r0 in range(0, rows, step):
        r1 = min(rows, r0 + step)
        out[r0:r1] = draw(rng, (r1 - r0, cols))
    return out


def uniform(rows: int, cols: int, seed: int, dtype=np.float32) -> np.ndarray:
    """i.i.d. uniform[-1, 1] entries."""
    rng = np.random.default_rng(seed)
    return _fill(rng, rows, cols, lambda g, s: g.uniform(-1.0, 1.0, s), dtype)


def normal(rows: int, cols: int, seed: int, dtype=np.float32) -> np.ndarray:
    """i.i.d. N(0, 1) entries."""
    rng = np.random.default_rng(seed)
    return _fill(rng, rows, cols, lambda g, s: g.standard_normal(s), dtype)


def scaled_normal(rows: int, cols: int, seed: int, dtype=np.float32,
                  span: float = 3.0) -> np.ndarray:
    """N(0, 1) entries with column j scaled by 10^u_j, u_j ~ U[-span, span].

    Draw order: the cols exponents u first, then the rows x cols normals.
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(-span, span, cols)
    scale = 10.0 ** u
    return _fill(rng, rows, cols, lambda g, s: g.standard_normal(s) * scale, dtype)


def sampled_columns(n: int, count: int, seed: int, after_rows: int = 0,
                    after_cols: int = 0) -> np.ndarray:
    """Sorted sample of ``count`` distinct column indices.

    For the 16384^2 precision workload the sample is drawn from the same
    Generator right after A; pass A's shape to reproduce that.
    """
    rng = np.random.default_rng(seed)
    if after_rows and after_cols:
        step = max(1, _CHUNK_ELEMS // after_cols)
        for r0 in range(0, after_rows, step):
            rng.standard_normal((min(after_rows, r0 + step) - r0, after_cols))
    return np.sort(rng.choice(n, count, replace=False)).astype(np.int64)


def batch_shapes(count: int = 512, seed: int = 5, m_range=(256, 8192),
                 n_range=(64, 2048)):
    """Log-uniform (m_i, n_i) for a batch of Gram products."""
    rng = np.random.default_rng(seed)
    m = np.rint(np.exp(rng.uniform(math.log(m_range[0]), math.log(m_range[1]), count)))
    n = np.rint(np.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1]), count)))
    return rng, m.astype(np.int64), n.astype(np.int64)


def batch(count: int = 512, seed: int = 5, m_range=(256, 8192), n_range=(64, 2048),
          dtype=np.float32):
    """List of uniform[-1,1] matrices with log-uniform shapes (shapes drawn first)."""
    rng, ms, ns = batch_shapes(count, seed, m_range, n_range)
    return [_fill(rng, int(m), int(n), lambda g, s: g.uniform(-1.0, 1.0, s), dtype)
            for m, n in zip(ms, ns)]


def make(name: str, rows: int | None = None, cols: int | None = None):
    """The named workload's matrix, optionally at a reduced shape."""
    w = WORKLOADS[name]
    r = rows if rows is not None else w.rows
    c = cols if cols is not None else w.cols
    dt = np.float64 if w.dtype == "f64" else np.float32
    if w.kind == "uniform":
        return uniform(r, c, w.seed, dt)
    if w.kind == "normal":
        return normal(r, c, w.seed, dt)
    if w.kind == "scaled_normal":
        return scaled_normal(r, c, w.seed, dt)
    raise ValueError("use batch() for the batched workload")
