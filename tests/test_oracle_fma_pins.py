"""Pins of the oracle's fused-multiply-add loops (the references of the
bitwise ONF parity) against their definition, in exact rational arithmetic.

The ONF kernel evaluates Eq. 3 (section "MoA Matrix Multiplication") in the
order of the paper's generic C program (section "From Normal Form to C
Program"): for each element, k ascending, one step c <- a*b + c per k. With
contraction, each step is the exact value a*b + c rounded once to the working
precision (IEEE 754 round to nearest, ties to even). The reference below
evaluates that step sequence with Fractions and its own rounding function, so
it shares nothing with the oracle's C loops; both oracle variants must match
it bit for bit. Copies of the C oracle with planted mistakes (unfused steps,
reversed k, a dropped last k) are built with gcc and must fail the pin.
"""
import ctypes
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "moa_oracle.c")

# binary64 / binary32: significand bits (with the hidden bit) and the least
# exponent of a normal number
FORMATS = {np.float64: (53, -1022), np.float32: (24, -126)}


def round_rne(x: Fraction, dtype) -> Fraction:
    """x rounded to the nearest value of `dtype`, ties to even (IEEE 754),
    for values inside the finite range."""
    if x == 0:
        return Fraction(0)
    prec, emin = FORMATS[dtype]
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()   # 2^e <= a < 2^(e+2)
    if Fraction(2) ** e > a:
        e -= 1
    if Fraction(2) ** (e + 1) <= a:
        e += 1
    quantum = Fraction(2) ** (max(e, emin) - (prec - 1))       # spacing of the grid around a
    q = a / quantum
    r = int(q)                                                 # floor for positive q
    rem = q - r
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and r % 2 == 1):
        r += 1
    v = r * quantum
    return v if x > 0 else -v


def to_float(v: Fraction, dtype):
    # exact: v is a value of dtype
    return dtype(float(v))


def fused_reference(A, B, dtype, k_order=None, fused=True):
    """Eq. 3 with one rounded step per k: c = RNE(a*b + c) when fused, else
    c = RNE(c + RNE(a*b)). k ascending unless k_order is given."""
    m, n = A.shape
    p = B.shape[1]
    ks = range(n) if k_order is None else k_order
    out = np.empty((m, p), dtype=dtype)
    Af = [[Fraction(float(A[i, k])) for k in range(n)] for i in range(m)]
    Bf = [[Fraction(float(B[k, j])) for j in range(p)] for k in range(n)]
    for i in range(m):
        for j in range(p):
            c = Fraction(0)
            for k in ks:
                prod = Af[i][k] * Bf[k][j]
                c = round_rne(prod + c, dtype) if fused else round_rne(c + round_rne(prod, dtype), dtype)
            out[i, j] = to_float(c, dtype)
    return out


def _operands(dtype, seed, m=4, n=40, p=5):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * 2.0 ** rng.integers(-6, 7, (m, n))
    B = rng.standard_normal((n, p))
    return A.astype(dtype), B.astype(dtype)


def test_round_rne_against_hand_values():
    """The rounding function itself, on values whose nearest neighbours are known."""
    one = Fraction(1)
    u32, u64 = Fraction(1, 2 ** 23), Fraction(1, 2 ** 52)
    # exact ties between 1 and 1 + ulp go to the even significand (1)
    assert round_rne(one + u32 / 2, np.float32) == one
    assert round_rne(one + u64 / 2, np.float64) == one
    # ties between 1 + ulp and 1 + 2 ulp go up to the even one (1 + 2 ulp)
    assert round_rne(one + 3 * u32 / 2, np.float32) == one + 2 * u32
    # just above a tie rounds up, just below rounds down
    assert round_rne(one + u32 / 2 + Fraction(1, 2 ** 60), np.float32) == one + u32
    assert round_rne(one + u32 / 2 - Fraction(1, 2 ** 60), np.float32) == one
    # 1/3 in binary32 and binary64 (known bit patterns)
    third = Fraction(1, 3)
    assert np.float32(float(round_rne(third, np.float32))).view(np.uint32) == 0x3EAAAAAB
    assert np.float64(float(round_rne(third, np.float64))).view(np.uint64) == 0x3FD5555555555555
    # subnormal grid of binary32: 2^-149 steps; half of it ties to zero (even)
    assert round_rne(Fraction(1, 2 ** 150), np.float32) == 0
    assert round_rne(Fraction(3, 2 ** 150), np.float32) == Fraction(2, 2 ** 149)
    assert round_rne(-third, np.float32) == -round_rne(third, np.float32)
    # agrees with the correctly rounded int/int division of Python for binary64
    rng = np.random.default_rng(0)
    for _ in range(500):
        x = Fraction(int(rng.integers(1, 2 ** 62)), int(rng.integers(1, 2 ** 62)))
        assert round_rne(x, np.float64) == Fraction(x.numerator / x.denominator)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_f32_fma_loop_is_the_fused_step_sequence(seed):
    A, B = _operands(np.float32, seed)
    ref = fused_reference(A, B, np.float32)
    assert np.array_equal(O.gemm_f32_fma(A, B).view(np.uint32), ref.view(np.uint32))
    # the pin discriminates: an unfused or reversed-k sequence gives other bits
    assert not np.array_equal(ref, fused_reference(A, B, np.float32, fused=False))
    assert not np.array_equal(ref, fused_reference(A, B, np.float32, k_order=range(A.shape[1] - 1, -1, -1)))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_f64_fma_loop_is_the_fused_step_sequence(seed):
    A, B = _operands(np.float64, seed)
    ref = fused_reference(A, B, np.float64)
    assert np.array_equal(O.gemm_f64_fma(A, B).view(np.uint64), ref.view(np.uint64))
    # and the unfused FP64 oracle is the unfused sequence
    assert np.array_equal(O.gemm_f64(A, B).view(np.uint64),
                          fused_reference(A, B, np.float64, fused=False).view(np.uint64))
    assert not np.array_equal(ref, fused_reference(A, B, np.float64, fused=False))


def test_f32_fma_accumulate_starts_from_given_c():
    A, B = _operands(np.float32, 5, m=3, n=12, p=4)
    C0 = np.random.default_rng(9).standard_normal((3, 4)).astype(np.float32)
    got = O.gemm_f32_fma(A, B, C0, accumulate=True)
    for i in range(3):
        for j in range(4):
            c = Fraction(float(C0[i, j]))
            for k in range(12):
                c = round_rne(Fraction(float(A[i, k])) * Fraction(float(B[k, j])) + c, np.float32)
            assert got[i, j] == np.float32(float(c))


# ------------------------------------------------------- planted mistakes --

PLANTS = {
    # an FP32 loop whose product is rounded before the add
    "f32_unfused": ("c_row[j] = fmaf(a, b_row[j], c_row[j]);", "c_row[j] = c_row[j] + a * b_row[j];"),
    # the FP32 k walk reversed
    "f32_reversed": (None, None),
    # the last k dropped from the FP32 walk
    "f32_drop_last": (None, None),
    "f64_unfused": ("c_row[j] = fma(a, b_row[j], c_row[j]);", "c_row[j] = c_row[j] + a * b_row[j];"),
    # the FP64 k walk reversed
    "f64_reversed": (None, None),
}


def _planted_source(kind):
    src = open(ORACLE_SRC).read()
    loops = {"f32_reversed": ("moa_oracle_gemm_f32_fma", "for (int64_t k = n - 1; k >= 0; --k)"),
             "f64_reversed": ("moa_oracle_gemm_f64_fma", "for (int64_t k = n - 1; k >= 0; --k)"),
             "f32_drop_last": ("moa_oracle_gemm_f32_fma", "for (int64_t k = 0; k < n - 1; ++k)")}
    if kind in loops:
        fn, loop = loops[kind]
        head, tail = src.split("void " + fn, 1)
        assert "for (int64_t k = 0; k < n; ++k)" in tail
        return head + "void " + fn + tail.replace("for (int64_t k = 0; k < n; ++k)", loop, 1)
    old, new = PLANTS[kind]
    assert src.count(old) == 1
    return src.replace(old, new)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("kind", sorted(PLANTS))
def test_planted_mistakes_fail_the_pin(kind):
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "planted.c")
        so = os.path.join(d, "planted.so")
        open(c, "w").write(_planted_source(kind))
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", c, "-o", so, "-lm"], check=True,
                       capture_output=True)
        lib = ctypes.CDLL(so)
        name = "moa_oracle_gemm_f32_fma" if kind.startswith("f32") else "moa_oracle_gemm_f64_fma"
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_void_p] * 3 + [ctypes.c_int]
        dt = np.float32 if kind.startswith("f32") else np.float64
        caught = False
        for seed in (0, 1, 2):
            A, B = _operands(dt, seed)
            out = np.empty((A.shape[0], B.shape[1]), dtype=dt)
            fn(A.shape[0], A.shape[1], B.shape[1], A.ctypes.data, B.ctypes.data, out.ctypes.data, 0)
            caught = caught or not np.array_equal(out, fused_reference(A, B, dt))
        assert caught, f"planted mistake {kind} passes the fused-step pin"
