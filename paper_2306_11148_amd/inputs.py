"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds random draws only: no part of the matrix product, its
number formats or its scaling rules lives here, so that both the CPU oracle
and the HIP library can be fed from it without sharing any of the method.

The paper names no dataset and no value distribution (its experiments are
square FP64 products up to 16000 x 16000 with unstated contents), so every
workload below is synthetic. All draws use numpy's PCG64 ``default_rng``.

Workloads (sizes and distributions fixed by the benchmark definitions):

* ``uniform_f64``      -- A, B i.i.d. uniform[-1, 1) in FP64 (256^3 case).
* ``integer_valued``   -- integers drawn uniformly from {-8, ..., 8}, stored as
                          FP64 or FP32; every partial sum is then exact.
* ``normal_f32``       -- A, B i.i.d. N(0, 1) rounded to FP32 (square sweep).
* ``row_col_scaled_f32`` -- N(0, 1) * 10^U(-3, 3) per row of A and per column
                          of B (wide dynamic range, precision study).
* ``grouped_shapes``   -- G shapes with m, n, p log-uniform in [lo, hi].
* ``serving_stream``   -- Poisson arrivals with log-uniform shapes and a
                          70/30 split-BF16 / FP8 path mix.
"""
from __future__ import annotations

import numpy as np


def uniform_f64(m: int, n: int, p: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1.0, 1.0, size=(m, n))
    B = rng.uniform(-1.0, 1.0, size=(n, p))
    return A, B


def integer_valued(m: int, n: int, p: int, seed: int = 0, dtype=np.float64):
    rng = np.random.default_rng(seed)
    A = rng.integers(-8, 9, size=(m, n)).astype(dtype)
    B = rng.integers(-8, 9, size=(n, p)).astype(dtype)
    return A, B


def normal_f32(m: int, n: int, p: int, seed: int):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal(size=(m, n), dtype=np.float32)
    B = rng.standard_normal(size=(n, p), dtype=np.float32)
    return A, B


def row_col_scaled_f32(m: int, n: int, p: int, seed: int = 3):
    rng = np.random.default_rng(seed)
    za = rng.standard_normal(size=(m, n))
    zb = rng.standard_normal(size=(n, p))
    u = rng.uniform(-3.0, 3.0, size=m)
    v = rng.uniform(-3.0, 3.0, size=p)
    A = (za * (10.0 ** u)[:, None]).astype(np.float32)
    B = (zb * (10.0 ** v)[None, :]).astype(np.float32)
    return A, B


def log_uniform_ints(rng, lo: int, hi: int, size):
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))).astype(np.int64)


def grouped_shapes(count: int = 512, lo: int = 32, hi: int = 2048, seed: int = 4):
    rng = np.random.default_rng(seed)
    return log_uniform_ints(rng, lo, hi, (count, 3))


def grouped_operands(shapes, seed: int = 4):
    """N(0,1) FP32 operands for each (m, n, p), drawn after the shapes."""
    rng = np.random.default_rng(seed + 1_000_003)
    out = []
    for m, n, p in shapes:
        A = rng.standard_normal(size=(int(m), int(n)), dtype=np.float32)
        B = rng.standard_normal(size=(int(n), int(p)), dtype=np.float32)
        out.append((A, B))
    return out


def serving_stream(count: int, rate_per_s: float, seed: int = 5,
                   mp_range=(64, 4096), n_range=(64, 8192), split_share=0.7):
    """Arrival times (s), shapes (count x 3) and a path flag (True = split-BF16)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    m = log_uniform_ints(rng, mp_range[0], mp_range[1], count)
    p = log_uniform_ints(rng, mp_range[0], mp_range[1], count)
    n = log_uniform_ints(rng, n_range[0], n_range[1], count)
    split = rng.uniform(size=count) < split_share
    return t, np.stack([m, n, p], axis=1), split


def operand_pool(elems: int, seed: int = 5):
    """One flat N(0,1) FP32 pool; a request's operand is a contiguous slice."""
    rng = np.random.default_rng(seed + 7)
    return rng.standard_normal(size=elems, dtype=np.float32)


def pool_offsets(rng_seed: int, count: int, sizes, pool_elems: int):
    rng = np.random.default_rng(rng_seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    return (rng.uniform(size=count) * (pool_elems - sizes + 1)).astype(np.int64)
