"""Operand layouts: gamma_row (default) and gamma_col for A, B and C.

A column-major operand is handed over as the transpose of a contiguous tensor
(logical shape unchanged; element (i, k) of the m x n matrix A at i + k m).

* Split-BF16 and FP8, every one of the 8 layout combinations, on ragged shapes:
  the path's bar against the oracle (split-BF16 <= 1e-5 against Eq. 3 in FP64,
  FP8 <= 1e-4 against the exact product of the quantised operands) and
  bit-exact on integer-valued inputs.
* ONF, every layout combination, FP64 and FP32, on ragged shapes: bitwise the
  fma-ordered oracle (a column-major operand is transposed on its way into the
  kernel's LDS slab; a column-major C runs as C^T = B^T A^T, and
  fma(b, a, c) = fma(a, b, c)). FP32 matrix cores, every combination: <= 1e-5
  against Eq. 3 and bit-exact on integers; the register-staged variant refuses
  a column-major operand.
* Grouped launches run members with a column-major operand singly: bitwise
  equal to moa_gemm.
"""
import itertools

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_11148_amd import inputs, moa

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
COMBOS = list(itertools.product([False, True], repeat=3))


def place(X, col):
    """Device tensor with the logical shape of X, row- or column-major."""
    if col:
        return torch.from_numpy(np.ascontiguousarray(X.T)).to(DEV).t()
    return torch.from_numpy(np.ascontiguousarray(X)).to(DEV)


def run(A, B, path, a_col, b_col, c_col, flags=0, dtype=np.float32):
    m, p = A.shape[0], B.shape[1]
    At, Bt = place(A, a_col), place(B, b_col)
    Ct = place(np.full((m, p), np.nan, dtype), c_col)
    d = moa.make_desc(At, Bt, Ct, path=path, flags=flags)
    # a column-major matrix with one row or column is also row-major (same memory)
    want = (moa.MOA_FLAG_A_COL if not At.is_contiguous() else 0) | \
        (moa.MOA_FLAG_B_COL if not Bt.is_contiguous() else 0) | (moa.MOA_FLAG_C_COL if not Ct.is_contiguous() else 0)
    assert d.flags & 0x7000000 == want
    assert want == (moa.MOA_FLAG_A_COL if a_col and min(A.shape) > 1 else 0) | \
        (moa.MOA_FLAG_B_COL if b_col and min(B.shape) > 1 else 0) | (moa.MOA_FLAG_C_COL if c_col and min(m, p) > 1 else 0)
    s = moa.lib().moa_gemm(__import__("ctypes").byref(d), None)
    if s != 0:
        raise moa.MoaError(s, "moa_gemm", moa.moa_last_error())
    torch.cuda.synchronize()
    return Ct.cpu().numpy()


@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("shape", [(129, 300, 77), (64, 1000, 200), (1, 50, 33)])
def test_split_bf16_every_layout(shape, combo):
    m, n, p = shape
    A, B = inputs.normal_f32(m, n, p, seed=m + n)
    C = run(A, B, "split_bf16", *combo)
    assert O.rel_err(C, O.gemm_f64(A.astype(np.float64), B.astype(np.float64))) <= 1e-5


@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("two", [False, True])
def test_fp8_every_layout(two, combo):
    A, B = inputs.row_col_scaled_f32(130, 700, 90, seed=22)
    C = run(A, B, "fp8", *combo, flags=moa.MOA_FLAG_FP8_TWO_TERM if two else moa.MOA_FLAG_FP8_ONE_TERM)
    Q = O.fp8_gemm_2term(A, B) if two else O.fp8_gemm(A, B)
    assert O.rel_err(C, Q) <= 1e-4


@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("path", ["split_bf16", "fp8"])
def test_every_layout_integer_exact(path, combo):
    A, B = inputs.integer_valued(70, 150, 50, seed=4, dtype=np.float32)
    C = run(A, B, path, *combo)
    assert np.array_equal(C.astype(np.float64), O.gemm_f64(A.astype(np.float64), B.astype(np.float64)))


@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("shape", [(200, 77, 333), (33, 130, 65), (1, 9, 130)])
def test_onf_every_layout_bitwise(shape, dt, combo):
    m, n, p = shape
    A, B = inputs.uniform_f64(m, n, p, seed=6 + m)
    A, B = A.astype(dt), B.astype(dt)
    C = run(A, B, "onf", *combo, dtype=dt)
    assert np.array_equal(C, O.gemm_f64_fma(A, B) if dt == np.float64 else O.gemm_f32_fma(A, B))


@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("shape", [(200, 300, 130), (65, 47, 300)])
def test_mfma_f32_every_layout(shape, combo):
    m, n, p = shape
    A, B = inputs.normal_f32(m, n, p, seed=7 + n)
    C = run(A, B, "mfma_f32", *combo)
    assert O.rel_err(C, O.gemm_f64(A.astype(np.float64), B.astype(np.float64))) <= 1e-5


@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("path", ["mfma_f32", "onf"])
def test_row_kernels_every_layout_integer_exact(path, combo):
    A, B = inputs.integer_valued(70, 150, 50, seed=5, dtype=np.float32)
    C = run(A, B, path, *combo)
    assert np.array_equal(C.astype(np.float64), O.gemm_f64(A.astype(np.float64), B.astype(np.float64)))


def test_register_staged_fp32_refuses_column_operands():
    A, B = inputs.normal_f32(20, 30, 40, seed=1)
    with pytest.raises(moa.MoaError) as ei:
        run(A, B, "mfma_f32", True, False, False, flags=moa.MOA_FLAG_VARIANT(2))
    assert ei.value.status == moa.MOA_ERR_UNSUPPORTED


def test_grouped_column_major_member_equals_single():
    shapes = [(90, 400, 70), (200, 300, 150), (64, 800, 64)]
    ops = inputs.grouped_operands(shapes, seed=19)
    cols = [(True, False, True), (False, False, False), (False, True, False)]
    descs, outs, refs = [], [], []
    for (A, B), (ac, bc, cc) in zip(ops, cols):
        At, Bt = place(A, ac), place(B, bc)
        Ct = place(np.zeros((A.shape[0], B.shape[1]), np.float32), cc)
        Rt = place(np.zeros((A.shape[0], B.shape[1]), np.float32), cc)
        moa.moa_gemm(At, Bt, Rt, path="split_bf16")
        descs.append(moa.make_desc(At, Bt, Ct, path="split_bf16"))
        outs.append((At, Bt, Ct))
        refs.append(Rt)
    moa.moa_gemm_grouped(descs)
    torch.cuda.synchronize()
    for (_, _, Ct), Rt in zip(outs, refs):
        assert torch.equal(Ct, Rt)
