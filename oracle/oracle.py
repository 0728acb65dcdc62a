"""CPU oracle for the MoA ONF matrix product and its reduced-precision paths.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. It shares no code
with the HIP library and never imports the ``paper_2306_11148_amd`` package.

Contents, each with the passage it follows:

* ``gemm_f64`` / ``gemm_f64_fma`` / ``gemm_f32_fma`` -- Eq. 3 of the section
  "MoA Matrix Multiplication", evaluated in the order of the paper's generic C
  program (section "From Normal Form to C Program"): row i, k ascending, the
  scalar A[i,k] times row k of B added into row i of C. The loops are plain C
  in ``moa_oracle.c`` (FP64, no multiply-add contraction; the *_fma variants
  use one fused multiply-add per step in the same order).
* ``static_block_components`` -- the block-size rule of section "Technical
  Details": three blocks (A, B, C) of b components of the element type must fit
  one per-processor memory budget; b is a power of two.
* ``bf16_split`` -- the 3-term BF16 split used by the split-BF16 path. The
  paper computes in FP64 and says nothing about reduced precision; this is the
  reading chosen for that path: hi = RNE_bf16(x), lo = RNE_bf16(x - hi), and
  the product is hi*hi + hi*lo + lo*hi (lo*lo dropped).
* ``e4m3_encode`` / ``e4m3_decode`` / ``pow2_exponents`` -- OCP FP8 E4M3
  (bias 7, 3 mantissa bits, largest finite 448, subnormal step 2^-9) with a
  per-row (A) / per-column (B) power-of-two scale 2^e, e the largest integer
  with amax * 2^e <= 448 (e = 0 for an all-zero row or column). The scales
  factor out of the k-sum, so C = 2^-(e_i+f_j) * sum_k qA[i,k] qB[k,j].

* ``hadamard`` / ``kronecker`` -- the Hadamard and Kronecker products the
  paper places with the matrix product in one family (ipophp, conclusion and
  appendix), written from their textbook definitions: C[i,j] = A[i,j] B[i,j];
  for A m x n and B p x q, C[i p + k, j q + l] = A[i,j] B[k,l]. Each element is
  one product rounded to the input precision; the accumulate form adds the
  rounded product to C with a second rounding (no fused multiply-add).
* ``gemm_batched`` -- a batch of independent products C[b] = A[b] B[b], the
  3-d contraction as "many parallel 2-d versions" (appendix).

Every function takes numpy arrays and returns numpy arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmoa_oracle.so")
_lib = None


def lib_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from oracle import build_oracle  # local build script, gcc only
        build_oracle.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64 = ctypes.c_int64
    vp = ctypes.c_void_p
    for name in ("moa_oracle_gemm_f64", "moa_oracle_gemm_f64_fma",
                 "moa_oracle_gemm_f32_fma"):
        fn = getattr(lib, name)
        fn.argtypes = [i64, i64, i64, vp, vp, vp, ctypes.c_int]
        fn.restype = None
    lib.moa_oracle_rel_err_f64.argtypes = [i64, vp, vp]
    lib.moa_oracle_rel_err_f64.restype = ctypes.c_double
    _lib = lib
    return lib


def _as(a, dtype, shape):
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.shape != shape:
        raise ValueError(f"shape {a.shape} != expected {shape}")
    return a


def _gemm(fn_name, dtype, A, B, C=None, accumulate=False):
    A = np.asarray(A)
    B = np.asarray(B)
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError(f"shapes {A.shape} x {B.shape} do not conform (Eq. 1)")
    m, n = A.shape
    p = B.shape[1]
    A = _as(A, dtype, (m, n))
    B = _as(B, dtype, (n, p))
    if accumulate:
        if C is None:
            raise ValueError("accumulate needs an initial C")
        out = np.array(C, dtype=dtype, copy=True, order="C")
        if out.shape != (m, p):
            raise ValueError("C shape")
    else:
        out = np.empty((m, p), dtype=dtype)
    if out.size:
        getattr(_load(), fn_name)(m, n, p, A.ctypes.data, B.ctypes.data,
                                  out.ctypes.data, int(bool(accumulate)))
    return out


def gemm_f64(A, B, C=None, accumulate=False):
    """Eq. 3 in FP64 (inputs widened exactly to FP64), product then add."""
    return _gemm("moa_oracle_gemm_f64", np.float64, A, B, C, accumulate)


def gemm_f64_fma(A, B, C=None, accumulate=False):
    """Eq. 3 in FP64, k ascending, fused multiply-add per step."""
    return _gemm("moa_oracle_gemm_f64_fma", np.float64, A, B, C, accumulate)


def gemm_f32_fma(A, B, C=None, accumulate=False):
    """Eq. 3 in FP32, k ascending, fused multiply-add per step."""
    A = np.asarray(A)
    B = np.asarray(B)
    if A.dtype != np.float32 or B.dtype != np.float32:
        raise TypeError("gemm_f32_fma takes float32 operands")
    return _gemm("moa_oracle_gemm_f32_fma", np.float32, A, B, C, accumulate)


def gemm_rows_f64(A, B, rows):
    """Rows ``rows`` of Eq. 3 in FP64 (row i of C depends only on row i of A)."""
    rows = np.asarray(rows, dtype=np.int64)
    return gemm_f64(np.asarray(A, dtype=np.float64)[rows], B)


def rel_err(X, R) -> float:
    """Normwise relative error ||X - R||_F / ||R||_F accumulated in FP64."""
    X = np.ascontiguousarray(X, dtype=np.float64).ravel()
    R = np.ascontiguousarray(R, dtype=np.float64).ravel()
    if X.shape != R.shape:
        raise ValueError("size mismatch")
    return float(_load().moa_oracle_rel_err_f64(X.size, X.ctypes.data,
                                                R.ctypes.data))


def max_row_rel_err(X, R) -> float:
    """Largest per-row relative error ||X_i - R_i||_2 / ||R_i||_2 (FP64)."""
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    worst = 0.0
    for i in range(R.shape[0]):
        d = np.sqrt(np.sum((X[i] - R[i]) ** 2))
        r = np.sqrt(np.sum(R[i] ** 2))
        worst = max(worst, d / r if r > 0 else d)
    return worst


# --------------------------------------------------------------------------
# Block-size rule (section "Technical Details")
# --------------------------------------------------------------------------

def static_block_components(budget_bytes: int, elem_bytes: int,
                            nblocks: int = 3) -> int:
    """Largest power of two b with nblocks * b * elem_bytes <= budget_bytes.

    The paper sizes one block each of A, B and C (three blocks) to one
    processor's memory and counts components, not the block's aspect ratio.
    Returns 0 if not even one component fits.
    """
    if budget_bytes <= 0 or elem_bytes <= 0 or nblocks <= 0:
        return 0
    b = 1
    if nblocks * b * elem_bytes > budget_bytes:
        return 0
    while nblocks * (2 * b) * elem_bytes <= budget_bytes:
        b *= 2
    return b


def block_shape(components: int) -> tuple[int, int]:
    """Squarest power-of-two shape (rows <= cols) with ``components`` entries."""
    if components <= 0 or components & (components - 1):
        raise ValueError("components must be a positive power of two")
    t = components.bit_length() - 1
    r = 1 << (t // 2)
    return r, components // r


# --------------------------------------------------------------------------
# BF16 split
# --------------------------------------------------------------------------

def bf16_round_bits(x32) -> np.ndarray:
    """BF16 code (uint16) nearest to each finite float32, ties to even.

    A BF16 value is the top 16 bits of a float32. Rounding to nearest even
    adds half an ulp minus one, plus the lowest kept bit, before truncating.
    """
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + keep_lsb) >> np.uint64(16)
    return (r & np.uint64(0xFFFF)).astype(np.uint16)


def bf16_to_f32(code) -> np.ndarray:
    c = np.ascontiguousarray(code, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return c.view(np.float32)


def bf16_split(x32):
    """(hi, lo) BF16 codes: hi = RNE(x), lo = RNE(x - hi); x - hi is exact."""
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    hi = bf16_round_bits(x32)
    resid = (x32.astype(np.float64) - bf16_to_f32(hi).astype(np.float64))
    resid32 = resid.astype(np.float32)
    if not np.array_equal(resid32.astype(np.float64), resid):
        raise AssertionError("x - hi not exact in float32")
    lo = bf16_round_bits(resid32)
    return hi, lo


def split_bf16_gemm(A32, B32):
    """FP64 value of hi_A hi_B + hi_A lo_B + lo_A hi_B (each term via Eq. 3)."""
    ah, al = (bf16_to_f32(t).astype(np.float64) for t in bf16_split(A32))
    bh, bl = (bf16_to_f32(t).astype(np.float64) for t in bf16_split(B32))
    return gemm_f64(ah, bh) + gemm_f64(ah, bl) + gemm_f64(al, bh)


# --------------------------------------------------------------------------
# OCP FP8 E4M3 with power-of-two row/column scaling
# --------------------------------------------------------------------------

E4M3_MAX = 448.0


def e4m3_decode(code) -> np.ndarray:
    """FP64 value of each E4M3 code (0x7F / 0xFF are NaN)."""
    c = np.asarray(code, dtype=np.uint8).astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    f = c & 0x7
    val = np.where(e == 0, f * 2.0 ** -9, (1.0 + f / 8.0) * np.exp2(e - 7.0))
    val = np.where((e == 15) & (f == 7), np.nan, val)
    return sign * val


def e4m3_encode(x) -> np.ndarray:
    """E4M3 code nearest to each finite value (ties to even), saturating at 448.

    Values below the smallest normal 2^-6 sit on the subnormal grid of step
    2^-9; a normal value with exponent E sits on the grid of step 2^(E-3).
    """
    x = np.asarray(x, dtype=np.float64)
    if not np.all(np.isfinite(x)):
        raise ValueError("finite inputs only")
    sign = np.signbit(x).astype(np.int64) << 7
    ax = np.abs(x)
    _, e2 = np.frexp(ax)                      # ax = f * 2^e2, f in [0.5, 1)
    E = e2.astype(np.int64) - 1               # ax in [2^E, 2^(E+1))
    sub = ax < 2.0 ** -6
    E = np.where(sub, -6, E)
    step = np.exp2((E - 3).astype(np.float64))
    q = np.rint(ax / step).astype(np.int64)   # numpy rint: ties to even
    # q in [0, 16]; on the subnormal grid q < 8 means exponent field 0.
    carry = q == 16
    E = np.where(carry, E + 1, E)
    q = np.where(carry, 8, q)
    normal = q >= 8
    field_e = np.where(normal, E + 7, 0)
    field_m = np.where(normal, q - 8, q)
    code = (field_e << 3) | field_m
    code = np.where(code > 0x7E, 0x7E, code)  # saturate to 448
    return (code | sign).astype(np.uint8)


def pow2_exponents(amax) -> np.ndarray:
    """Largest integer e with amax * 2^e <= 448; 0 where amax == 0."""
    amax = np.asarray(amax, dtype=np.float64)
    f, E = np.frexp(amax)                     # amax = f * 2^E, f in [0.5, 1)
    # 448 = 0.875 * 2^9, so f * 2^(E+e) <= 0.875 * 2^9 decides e exactly.
    e = np.where(f <= 0.875, 9 - E, 8 - E).astype(np.int64)
    return np.where(amax == 0, 0, e)


def fp8_quantise(A32, B32):
    """(qA codes, e per row of A, qB codes, f per column of B)."""
    A = np.asarray(A32, dtype=np.float32).astype(np.float64)
    B = np.asarray(B32, dtype=np.float32).astype(np.float64)
    e = pow2_exponents(np.abs(A).max(axis=1) if A.shape[1] else np.zeros(A.shape[0]))
    f = pow2_exponents(np.abs(B).max(axis=0) if B.shape[0] else np.zeros(B.shape[1]))
    qA = e4m3_encode(A * np.exp2(e.astype(np.float64))[:, None])
    qB = e4m3_encode(B * np.exp2(f.astype(np.float64))[None, :])
    return qA, e, qB, f


def fp8_gemm(A32, B32):
    """FP64 value of the 1-term scaled-FP8 product 2^-(e_i+f_j) sum_k qA qB."""
    qA, e, qB, f = fp8_quantise(A32, B32)
    acc = gemm_f64(e4m3_decode(qA), e4m3_decode(qB))
    return acc * np.exp2(-(e[:, None] + f[None, :]).astype(np.float64))


LO_SHIFT = 4   # the FP8 residual term is stored pre-multiplied by 2^4


def fp8_quantise_2term(A32, B32):
    """2-term FP8: hi codes as in ``fp8_quantise``; lo = E4M3(2^4 (x 2^e - hi))."""
    qA, e, qB, f = fp8_quantise(A32, B32)
    A = np.asarray(A32, dtype=np.float32).astype(np.float64) * np.exp2(e.astype(np.float64))[:, None]
    B = np.asarray(B32, dtype=np.float32).astype(np.float64) * np.exp2(f.astype(np.float64))[None, :]
    lA = e4m3_encode((A - e4m3_decode(qA)) * 2.0 ** LO_SHIFT)
    lB = e4m3_encode((B - e4m3_decode(qB)) * 2.0 ** LO_SHIFT)
    return qA, lA, e, qB, lB, f


def fp8_gemm_2term(A32, B32):
    """FP64 value of 2^-(e_i+f_j) [hA hB + 2^-4 (hA lB + lA hB)]."""
    qA, lA, e, qB, lB, f = fp8_quantise_2term(A32, B32)
    hA, hB = e4m3_decode(qA), e4m3_decode(qB)
    acc = gemm_f64(hA, hB) + 2.0 ** -LO_SHIFT * (gemm_f64(hA, e4m3_decode(lB)) +
                                                  gemm_f64(e4m3_decode(lA), hB))
    return acc * np.exp2(-(e[:, None] + f[None, :]).astype(np.float64))


# ---------------------------------------------------------------- ipophp --

def _round_to(x64, dtype):
    """FP64 values rounded once to `dtype` (FP64 holds every FP32 product and
    sum of two FP32 values exactly or with innocuous double rounding)."""
    return np.asarray(x64, dtype=np.float64).astype(dtype)


def hadamard(A, B, C=None, accumulate=False):
    """C[i,j] := A[i,j] * B[i,j] (or C[i,j] + that product), in A's precision."""
    A = np.asarray(A)
    dt = A.dtype
    P = _round_to(A.astype(np.float64) * np.asarray(B, dtype=np.float64), dt)
    if not accumulate:
        return P
    return _round_to(P.astype(np.float64) + np.asarray(C, dtype=np.float64), dt)


def kronecker(A, B, C=None, accumulate=False):
    """A (m x n), B (p x q) -> C ((m p) x (n q)) with C[i p + k, j q + l] =
    A[i,j] B[k,l]: block (i, j) of C is A[i,j] times B."""
    A = np.asarray(A)
    B = np.asarray(B)
    dt = A.dtype
    m, n = A.shape
    p, q = B.shape
    B64 = B.astype(np.float64)
    out = np.empty((m * p, n * q), dtype=dt)
    for i in range(m):
        for j in range(n):
            blk = _round_to(float(A[i, j]) * B64, dt)
            if accumulate:
                blk = _round_to(blk.astype(np.float64) + np.asarray(C, dtype=np.float64)[i * p:(i + 1) * p,
                                                                                          j * q:(j + 1) * q], dt)
            out[i * p:(i + 1) * p, j * q:(j + 1) * q] = blk
    return out


def gemm_batched(A, B):
    """C[b] = A[b] B[b] (Eq. 3 per member, FP64) for 3-d arrays A (batch x m x n)
    and B (batch x n x p)."""
    return np.stack([gemm_f64(np.asarray(A[b], dtype=np.float64), np.asarray(B[b], dtype=np.float64))
                     for b in range(len(A))])
