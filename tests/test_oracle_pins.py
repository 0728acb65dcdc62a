"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Eq. 3 (section "MoA Matrix Multiplication") is checked against exact rational
arithmetic, closed forms, identity/permutation/diagonal products, the
transpose law, linearity, the textbook row-column loop (bitwise), and the
dimension-lifting invariance of section "Dimension Lifting to Machine
Coordinates". The number formats are checked against published format facts
(tests/golden/number_formats.json) and torch's own casts. The block-size rule
is pinned by the numbers of section "Technical Details"
(tests/golden/static_rule_paper.json).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_11148_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2.0 ** -53


def exact_product(A, B):
    m, n = A.shape
    p = B.shape[1]
    Af = [[Fraction(float(A[i, k])) for k in range(n)] for i in range(m)]
    Bf = [[Fraction(float(B[k, j])) for j in range(p)] for k in range(n)]
    return [[sum((Af[i][k] * Bf[k][j] for k in range(n)), Fraction(0))
             for j in range(p)] for i in range(m)]


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 2), (4, 8, 7), (7, 3, 8), (2, 16, 3)])
@pytest.mark.parametrize("fn", [O.gemm_f64, O.gemm_f64_fma])
def test_exact_rational_within_dot_product_bound(shape, fn):
    """|R - AB| <= gamma_n |A||B| elementwise (Higham, dot-product bound)."""
    m, n, p = shape
    rng = np.random.default_rng(sum(shape))
    A = rng.uniform(-1, 1, (m, n)) * 10.0 ** rng.uniform(-3, 3, (m, n))
    B = rng.uniform(-1, 1, (n, p))
    R = fn(A, B)
    X = exact_product(A, B)
    gamma = n * U64 / (1 - n * U64)
    absAB = np.abs(A) @ np.abs(B)
    for i in range(m):
        for j in range(p):
            err = abs(Fraction(float(R[i, j])) - X[i][j])
            assert err <= Fraction(gamma * absAB[i, j]) * (1 + Fraction(1, 10**6))


def test_fma_variant_differs_from_unfused_somewhere():
    """The two FP64 variants must really be different operation sequences."""
    A, B = inputs.uniform_f64(32, 64, 32, seed=11)
    assert not np.array_equal(O.gemm_f64(A, B), O.gemm_f64_fma(A, B))


def test_textbook_row_column_loop_bitwise():
    """i-j-k dot products (Python floats: IEEE double, no contraction)."""
    A, B = inputs.uniform_f64(6, 9, 5, seed=3)
    R = O.gemm_f64(A, B)
    for i in range(6):
        for j in range(5):
            s = 0.0
            for k in range(9):
                s = s + float(A[i, k]) * float(B[k, j])
            assert s == R[i, j]


def test_closed_forms():
    m, n, p = 5, 37, 6
    assert np.all(O.gemm_f64(np.ones((m, n)), np.ones((n, p))) == n)
    Ak = np.tile(np.arange(n, dtype=np.float64), (m, 1))      # A[i, k] = k
    assert np.all(O.gemm_f64(Ak, np.ones((n, p))) == n * (n - 1) / 2)
    Bk = np.tile(np.arange(n, dtype=np.float64)[:, None], (1, p))  # B[k, j] = k
    Bk = Bk * (np.arange(p) + 1)[None, :]                      # B[k, j] = k (j+1)
    assert np.array_equal(O.gemm_f64(np.ones((m, n)), Bk),
                          np.tile((n * (n - 1) / 2) * (np.arange(p) + 1.0), (m, 1)))
    f32 = O.gemm_f32_fma(np.ones((m, n), np.float32), np.ones((n, p), np.float32))
    assert f32.dtype == np.float32 and np.all(f32 == n)


def test_identity_permutation_diagonal():
    rng = np.random.default_rng(1)
    A = rng.uniform(-1, 1, (7, 5))
    B = rng.uniform(-1, 1, (5, 9))
    assert np.array_equal(O.gemm_f64(A, np.eye(5)), A)
    assert np.array_equal(O.gemm_f64(np.eye(5), B), B)
    perm = rng.permutation(5)
    P = np.eye(5)[perm]                                        # (P B)[r] = B[perm[r]]
    assert np.array_equal(O.gemm_f64(P, B), B[perm])
    Q = np.eye(9)[:, perm_cols := rng.permutation(9)]          # (B Q)[:, c] = B[:, perm[c]]
    assert np.array_equal(O.gemm_f64(B, Q), B[:, perm_cols])
    d = 2.0 ** rng.integers(-4, 5, 7)
    assert np.array_equal(O.gemm_f64(np.diag(d), A), A * d[:, None])


def test_transpose_law_bitwise():
    """(AB)^T = B^T A^T: same products, same ascending k order."""
    A, B = inputs.uniform_f64(11, 13, 7, seed=5)
    assert np.array_equal(O.gemm_f64(A, B).T, O.gemm_f64(B.T.copy(), A.T.copy()))
    A32, B32 = inputs.normal_f32(9, 17, 6, seed=6)
    assert np.array_equal(O.gemm_f32_fma(A32, B32).T,
                          O.gemm_f32_fma(B32.T.copy(), A32.T.copy()))


def test_linearity_integer_valued():
    A, B = inputs.integer_valued(8, 21, 10, seed=2)
    A2, _ = inputs.integer_valued(8, 21, 10, seed=9)
    lhs = O.gemm_f64(4.0 * A - 0.5 * A2, B)
    rhs = 4.0 * O.gemm_f64(A, B) - 0.5 * O.gemm_f64(A2, B)
    assert np.array_equal(lhs, rhs)


def test_accumulate_and_empty_dimensions():
    A, B = inputs.integer_valued(4, 6, 3, seed=4)
    C0 = np.arange(12, dtype=np.float64).reshape(4, 3)
    assert np.array_equal(O.gemm_f64(A, B, C0, accumulate=True), C0 + O.gemm_f64(A, B))
    # n = 0: the empty sum assigns zero, or leaves C when accumulating
    Z = O.gemm_f64(np.zeros((4, 0)), np.zeros((0, 3)))
    assert Z.shape == (4, 3) and np.all(Z == 0)
    assert np.array_equal(O.gemm_f64(np.zeros((4, 0)), np.zeros((0, 3)), C0, True), C0)
    assert O.gemm_f64(np.zeros((0, 5)), np.zeros((5, 3))).shape == (0, 3)
    assert O.gemm_f64(np.zeros((2, 5)), np.zeros((5, 0))).shape == (2, 0)
    with pytest.raises(ValueError):
        O.gemm_f64(np.zeros((2, 5)), np.zeros((4, 3)))


def test_row_and_column_lifting_is_bitwise_invariant():
    """Splitting i over 'processors' or j over register groups keeps results."""
    A, B = inputs.uniform_f64(12, 19, 24, seed=8)
    R = O.gemm_f64(A, B)
    for nproc in (1, 2, 3, 4, 12):
        rows = 12 // nproc
        parts = [O.gemm_f64(A[q * rows:(q + 1) * rows], B) for q in range(nproc)]
        assert np.array_equal(np.vstack(parts), R)
    for rsize in (1, 3, 8, 24):
        parts = [O.gemm_f64(A, B[:, g * rsize:(g + 1) * rsize].copy()) for g in range(24 // rsize)]
        assert np.array_equal(np.hstack(parts), R)
    assert np.array_equal(O.gemm_rows_f64(A, B, [3, 0, 11]), R[[3, 0, 11]])


def test_numpy_matmul_within_bound():
    A, B = inputs.uniform_f64(64, 200, 48, seed=13)
    R = O.gemm_f64(A, B)
    gamma = 200 * U64 / (1 - 200 * U64)
    assert np.all(np.abs(R - A @ B) <= 2 * gamma * (np.abs(A) @ np.abs(B)))


def test_f32_fma_matches_f64_on_integers_and_bound_on_random():
    A, B = inputs.integer_valued(16, 300, 9, seed=1, dtype=np.float32)
    assert np.array_equal(O.gemm_f32_fma(A, B).astype(np.float64),
                          O.gemm_f64(A.astype(np.float64), B.astype(np.float64)))
    A, B = inputs.normal_f32(16, 300, 9, seed=2)
    R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
    u32 = 2.0 ** -24
    gamma = 300 * u32 / (1 - 300 * u32)
    assert np.all(np.abs(O.gemm_f32_fma(A, B) - R) <=
                  gamma * (np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))))


def test_rel_err_definition():
    R = np.array([[3.0, 4.0]])
    assert O.rel_err(R, R) == 0.0
    assert O.rel_err(np.array([[3.0, 4.0 + 5.0]]), R) == 1.0
    assert O.rel_err(np.array([[0.0, 0.0]]), R) == 1.0


# --------------------------------------------------------------------------
# Block-size rule
# --------------------------------------------------------------------------

def test_static_rule_reproduces_paper_numbers():
    g = json.load(open(os.path.join(GOLDEN, "static_rule_paper.json")))
    for c in g["cases"]:
        b = O.static_block_components(c["budget_bytes"], c["elem_bytes"], c["nblocks"])
        assert b == c["components"]
        assert b * c["elem_bytes"] == c["block_bytes"]
        assert 3 * b * c["elem_bytes"] == c["three_block_bytes"]
        for r, s in c["equivalent_shapes"]:
            assert r * s == b
    assert O.block_shape(1024) == (32, 32)
    assert O.block_shape(2048) == (32, 64)
    assert O.static_block_components(23, 8) == 0


# --------------------------------------------------------------------------
# Number formats
# --------------------------------------------------------------------------

def _formats():
    return json.load(open(os.path.join(GOLDEN, "number_formats.json")))


def test_bf16_split_golden():
    for c in _formats()["bf16_cases"]:
        x = np.array([int(c["x_hex"], 16)], dtype=np.uint32).view(np.float32)
        hi, lo = O.bf16_split(x)
        assert f"{hi[0]:04x}" == c["hi"], c["why"]
        assert f"{lo[0]:04x}" == c["lo"], c["why"]


def test_bf16_rounding_matches_torch_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(200_000).astype(np.float32),
        (rng.standard_normal(50_000) * 10.0 ** rng.uniform(-30, 30, 50_000)).astype(np.float32),
        # exact ties: low 16 bits == 0x8000
        (rng.integers(0, 2**31, 20_000, dtype=np.uint32) & np.uint32(0xFFFF0000) |
         np.uint32(0x8000)).view(np.float32),
    ])
    x = x[np.isfinite(x) & (np.abs(x) < 3e38)]
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(O.bf16_round_bits(x), ref)


def test_bf16_split_reconstruction():
    A, _ = inputs.row_col_scaled_f32(64, 64, 1, seed=3)
    hi, lo = O.bf16_split(A)
    h = O.bf16_to_f32(hi).astype(np.float64)
    lo_v = O.bf16_to_f32(lo).astype(np.float64)
    x = A.astype(np.float64)
    assert np.all(np.abs(x - h) <= 2.0 ** -8 * np.abs(x))          # hi: 8 significant bits
    assert np.all(np.abs(x - h - lo_v) <= 2.0 ** -16 * np.abs(x))  # hi + lo: 16 bits
    Ai, _ = inputs.integer_valued(8, 8, 1, seed=1, dtype=np.float32)
    hi, lo = O.bf16_split(Ai)
    assert np.all(lo == 0) and np.array_equal(O.bf16_to_f32(hi), Ai)


def test_e4m3_decode_golden_and_torch():
    for c in _formats()["e4m3_decode"]:
        assert O.e4m3_decode(np.array([int(c["code"], 16)]))[0] == c["value"]
    codes = np.arange(256, dtype=np.uint8)
    ours = O.e4m3_decode(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).double().numpy()
    finite = ~np.isnan(ref)
    assert np.array_equal(np.isnan(ours), ~finite)
    assert np.array_equal(ours[finite], ref[finite])


def test_e4m3_encode_golden():
    for c in _formats()["e4m3_encode"]:
        assert f"{O.e4m3_encode(np.array([c['x']]))[0]:02x}" == c["code"], c["why"]


def test_e4m3_encode_matches_torch_cast_including_ties():
    vals = O.e4m3_decode(np.arange(256, dtype=np.uint8))
    grid = np.unique(vals[np.isfinite(vals)])
    mids = (grid[:-1] + grid[1:]) / 2.0                 # exact ties
    rng = np.random.default_rng(7)
    rand = rng.uniform(-448, 448, 100_000) * 2.0 ** rng.integers(-14, 1, 100_000)
    x = np.concatenate([grid, mids, rand]).astype(np.float32)
    ours = O.e4m3_encode(x.astype(np.float64))
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)


def test_pow2_exponent_rule():
    for c in _formats()["pow2_exponent_cases"]:
        assert O.pow2_exponents(np.array([c["amax"]]))[0] == c["e"], c
    rng = np.random.default_rng(3)
    amax = rng.uniform(0.1, 1.0, 10_000) * 10.0 ** rng.uniform(-20, 20, 10_000)
    e = O.pow2_exponents(amax).astype(np.float64)
    assert np.all(amax * 2.0 ** e <= 448.0)
    assert np.all(amax * 2.0 ** (e + 1) > 448.0)


def test_reduced_precision_products_exact_on_integers():
    """Small integers are exact in BF16 (lo = 0) and, scaled, in E4M3."""
    A, B = inputs.integer_valued(12, 40, 10, seed=5, dtype=np.float32)
    R = O.gemm_f64(A, B)
    assert np.array_equal(O.split_bf16_gemm(A, B), R)
    assert np.array_equal(O.fp8_gemm(A, B), R)
    assert np.array_equal(O.fp8_gemm_2term(A, B), R)


def test_fp8_scales_follow_rows_of_A_and_columns_of_B():
    """Rows of A and columns of B carry different powers of two; only the
    per-row (A) / per-column (B) scaling keeps every entry exact."""
    A, B = inputs.integer_valued(6, 10, 7, seed=8, dtype=np.float32)
    ra = 2.0 ** np.arange(-9, 9, 3)                    # 6 rows
    cb = 2.0 ** np.arange(12, -16, -4)                 # 7 columns
    As = (A * ra[:, None]).astype(np.float32)
    Bs = (B * cb[None, :]).astype(np.float32)
    R = O.gemm_f64(As.astype(np.float64), Bs.astype(np.float64))
    assert np.array_equal(O.fp8_gemm(As, Bs), R)
    qA, e, qB, f = O.fp8_quantise(As, Bs)
    assert np.all(np.abs(O.e4m3_decode(qA)) <= 448) and np.all(np.abs(O.e4m3_decode(qB)) <= 448)
    amaxA = np.abs(As).max(axis=1).astype(np.float64)
    assert np.all(amaxA * 2.0 ** e <= 448) and np.all(amaxA * 2.0 ** (e + 1) > 448)


def test_reduced_precision_error_levels():
    """Measured errors of the reduced-precision readings versus Eq. 3 in FP64."""
    A, B = inputs.normal_f32(48, 512, 40, seed=21)
    R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
    e_split = O.rel_err(O.split_bf16_gemm(A, B), R)
    e_fp8 = O.rel_err(O.fp8_gemm(A, B), R)
    e_fp8_2 = O.rel_err(O.fp8_gemm_2term(A, B), R)
    assert e_split < 1e-5
    assert 1e-2 < e_fp8 < 6e-2          # 4 significant bits per operand
    assert e_fp8_2 < 3e-3


# ------------------------------------------------- ipophp family (f3) --

def test_kronecker_golden_hand_values():
    g = json.load(open(os.path.join(GOLDEN, "kronecker_small.json")))
    for a, b, c in (("A", "B", "C"), ("A2", "B2", "C2")):
        A = np.array(g[a], np.float64)
        B = np.array(g[b], np.float64)
        assert np.array_equal(O.kronecker(A, B), np.array(g[c], np.float64))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_kronecker_matches_library_and_identities(dt):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((3, 4)).astype(dt)
    B = rng.standard_normal((5, 2)).astype(dt)
    assert np.array_equal(O.kronecker(A, B), np.kron(A, B))
    # transpose: (A (x) B)^T = A^T (x) B^T
    assert np.array_equal(O.kronecker(A, B).T, O.kronecker(A.T.copy(), B.T.copy()))
    # mixed product on integers (exact): (A (x) B)(C (x) D) = (AC) (x) (BD)
    Ai = rng.integers(-3, 4, (2, 3)).astype(np.float64)
    Bi = rng.integers(-3, 4, (3, 2)).astype(np.float64)
    Ci = rng.integers(-3, 4, (3, 2)).astype(np.float64)
    Di = rng.integers(-3, 4, (2, 4)).astype(np.float64)
    lhs = O.gemm_f64(O.kronecker(Ai, Bi), O.kronecker(Ci, Di))
    rhs = O.kronecker(O.gemm_f64(Ai, Ci), O.gemm_f64(Bi, Di))
    assert np.array_equal(lhs, rhs)
    # identity (x) B is block diagonal
    K = O.kronecker(np.eye(3, dtype=dt), B)
    for i in range(3):
        for j in range(3):
            blk = K[i * 5:(i + 1) * 5, j * 2:(j + 1) * 2]
            assert np.array_equal(blk, B if i == j else np.zeros_like(B))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_hadamard_matches_library_and_accumulate_rounding(dt):
    rng = np.random.default_rng(6)
    A = rng.standard_normal((7, 9)).astype(dt)
    B = rng.standard_normal((7, 9)).astype(dt)
    C = rng.standard_normal((7, 9)).astype(dt)
    assert np.array_equal(O.hadamard(A, B), np.multiply(A, B))
    assert np.array_equal(O.hadamard(A, B), O.hadamard(B, A))
    # accumulate = two roundings in the input precision (numpy's own arithmetic)
    assert np.array_equal(O.hadamard(A, B, C, accumulate=True), (A * B) + C)
    K = O.kronecker(A[:2, :3], B[:3, :2], O.kronecker(A[:2, :3], B[:3, :2]), accumulate=True)
    assert np.array_equal(K, np.kron(A[:2, :3], B[:3, :2]) * dt(2))


def test_gemm_batched_members():
    rng = np.random.default_rng(7)
    A = rng.integers(-8, 9, (3, 4, 5)).astype(np.float64)
    B = rng.integers(-8, 9, (3, 5, 6)).astype(np.float64)
    assert np.array_equal(O.gemm_batched(A, B), np.matmul(A, B))


def test_max_row_rel_err_hand_values():
    """Largest per-row error ||X_i - R_i|| / ||R_i|| (rows of C3 span 10^+-3,
    where a normwise figure is dominated by the largest rows)."""
    R = np.array([[3.0, 4.0], [0.0, 1e-3], [1e3, 0.0]])
    X = np.array([[3.0, 4.0], [0.0, 2e-3], [1e3 + 1.0, 0.0]])
    # row 0 exact, row 1 off by 100%, row 2 off by 1e-3
    assert O.max_row_rel_err(X, R) == pytest.approx(1.0, rel=1e-15)
    assert O.max_row_rel_err(X[[0, 2]], R[[0, 2]]) == pytest.approx(1e-3, rel=1e-12)
    # the normwise error of the same data hides the small row
    assert O.rel_err(X, R) < 2e-3
    # a zero row of R contributes its absolute error
    assert O.max_row_rel_err(np.array([[0.0, 0.5]]), np.zeros((1, 2))) == 0.5
    assert O.max_row_rel_err(R, R) == 0.0
