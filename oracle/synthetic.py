"""Counter-based synthetic operands of the serving workload, CPU side.

TEST INFRASTRUCTURE. Only the test suite and the ``cpu_baseline`` leg of
``bench.py`` may import this module. The HIP library draws the same operands
on the device with its own implementation of the same published generator;
the two share no code.

The serving workload's requests are (shape, path, seed) and their operands
are generated where they are used, so the CPU side cannot be handed the
device's draws: each side implements the generator from its definition.

* ``philox4x32_10`` -- Philox4x32 with 10 rounds (Salmon, Moraes, Dror and
  Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011, section 4):
  a 128-bit counter (four 32-bit words c0..c3) and a 64-bit key (k0, k1).
  One round multiplies c0 by 0xD2511F53 and c2 by 0xCD9E8D57 into 64-bit
  products and forms (hi(c2 M1) ^ c1 ^ k0, lo(c2 M1), hi(c0 M0) ^ c3 ^ k1,
  lo(c0 M0)); between rounds the key is bumped by the Weyl constants
  (0x9E3779B9, 0xBB67AE85), all modulo 2^32.
* ``synthetic_operand`` -- element e (row-major flat index) of operand `tag`
  (0 = A, 1 = B) of a request with 64-bit `seed`: pair q = e div 2 draws one
  Philox block with counter (q mod 2^32, q div 2^32, tag, 0) and key
  (seed mod 2^32, seed div 2^32); element 2q takes words x0, x1 and element
  2q+1 words x2, x3. With S the sum of the four 16-bit halves of its two
  words, the value is the FP32 product (2 S - 4 * 65535) * c, c the FP32
  value nearest sqrt(3) * 2^-17: a scaled sum of four uniform variates
  (Irwin-Hall), symmetric about 0 with unit variance, in [-3.4641, 3.4641].
  2 S - 4 * 65535 is an integer of at most 19 bits, so the only rounding is
  that one FP32 multiplication.
"""
from __future__ import annotations

import numpy as np

PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = 0xFFFFFFFF
SCALE = np.float32(np.sqrt(3.0) / 131072.0)


def _mulhilo(a: int, x: np.ndarray):
    prod = np.uint64(a) * x.astype(np.uint64)
    return (prod >> np.uint64(32)).astype(np.uint32), (prod & np.uint64(MASK32)).astype(np.uint32)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox4x32 rounds over arrays of counters (uint32), one key."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint32) for x in (c0, c1, c2, c3))
    k0, k1 = int(k0) & MASK32, int(k1) & MASK32
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        hi0, lo0 = _mulhilo(PHILOX_M0, c0)
        hi1, lo1 = _mulhilo(PHILOX_M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint32(k0), lo1, hi0 ^ c3 ^ np.uint32(k1), lo0
    return c0, c1, c2, c3


def _halves_sum(w0, w1):
    s = (w0 & np.uint32(0xFFFF)).astype(np.int64) + (w0 >> np.uint32(16)).astype(np.int64)
    return s + (w1 & np.uint32(0xFFFF)).astype(np.int64) + (w1 >> np.uint32(16)).astype(np.int64)


def synthetic_elements(idx, seed: int, tag: int) -> np.ndarray:
    """FP32 values of the elements with flat indices `idx` (any int array)."""
    idx = np.asarray(idx, dtype=np.int64)
    q = idx >> 1
    x0, x1, x2, x3 = philox4x32_10((q & MASK32).astype(np.uint32), (q >> 32).astype(np.uint32),
                                   np.full(q.shape, tag, dtype=np.uint32), np.zeros(q.shape, dtype=np.uint32),
                                   seed & MASK32, (seed >> 32) & MASK32)
    odd = (idx & 1).astype(bool)
    s = np.where(odd, _halves_sum(x2, x3), _halves_sum(x0, x1))
    return (2 * s - 4 * 65535).astype(np.float32) * SCALE


def synthetic_range(start: int, count: int, seed: int, tag: int) -> np.ndarray:
    """Elements start .. start + count - 1 (FP32), one generator block per pair."""
    if count <= 0:
        return np.zeros(0, dtype=np.float32)
    q0, q1 = start >> 1, (start + count - 1) >> 1
    q = np.arange(q0, q1 + 1, dtype=np.int64)
    x0, x1, x2, x3 = philox4x32_10((q & MASK32).astype(np.uint32), (q >> 32).astype(np.uint32),
                                   np.full(q.shape, tag, dtype=np.uint32), np.zeros(q.shape, dtype=np.uint32),
                                   seed & MASK32, (seed >> 32) & MASK32)
    s = np.empty(2 * q.size, dtype=np.int64)
    s[0::2] = _halves_sum(x0, x1)
    s[1::2] = _halves_sum(x2, x3)
    first = start - 2 * q0
    return (2 * s[first:first + count] - 4 * 65535).astype(np.float32) * SCALE


def synthetic_operand(rows: int, cols: int, seed: int, tag: int, row_index=None) -> np.ndarray:
    """The rows x cols row-major operand `tag` of a request (FP32); with
    `row_index`, only those rows (in that order)."""
    if row_index is None:
        return synthetic_range(0, rows * cols, seed, tag).reshape(rows, cols)
    out = np.empty((len(row_index), cols), dtype=np.float32)
    for k, r in enumerate(row_index):
        out[k] = synthetic_range(int(r) * cols, cols, seed, tag)
    return out
