"""Split-k (the sigma-lift across workgroups, Fig. 2's addition loop over k
blocks) on the split-BF16 and FP8 paths.

* Skinny and ragged shapes meet each path's bar against the oracle: split-BF16
  <= 1e-5 normwise against Eq. 3 in FP64, FP8 <= 1e-4 against the exact product
  of the quantised operands.
* Integer-valued inputs stay bit-exact (every partial sum is an exact integer).
* The chunk partials are added in a fixed order: two runs give the same bits.
* A grouped launch runs a split-k member as a single launch: bitwise equal to
  moa_gemm on the same descriptor. Prepared groups refuse such members.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_11148_amd import inputs, moa

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def run(A, B, path, flags, accumulate=False, C0=None):
    At = torch.from_numpy(np.ascontiguousarray(A)).to(DEV)
    Bt = torch.from_numpy(np.ascontiguousarray(B)).to(DEV)
    m, p = A.shape[0], B.shape[1]
    Ct = (torch.from_numpy(C0).to(DEV) if C0 is not None
          else torch.full((m, p), float("nan"), device=DEV))
    moa.moa_gemm(At, Bt, Ct, path=path, accumulate=accumulate, flags=flags)
    torch.cuda.synchronize()
    return Ct.cpu().numpy()


SHAPES = [(100, 20000, 100), (257, 5000, 129), (1, 3000, 300), (33, 70, 17)]


@pytest.mark.parametrize("chunks", [2, 7, 32])
@pytest.mark.parametrize("shape", SHAPES)
def test_split_bf16_split_k_tolerance_and_determinism(shape, chunks):
    m, n, p = shape
    A, B = inputs.normal_f32(m, n, p, seed=m + n + chunks)
    fl = moa.MOA_FLAG_SPLIT_K(chunks)
    C = run(A, B, "split_bf16", fl)
    assert O.rel_err(C, O.gemm_f64(A.astype(np.float64), B.astype(np.float64))) <= 1e-5
    assert np.array_equal(C, run(A, B, "split_bf16", fl))


@pytest.mark.parametrize("two", [False, True])
@pytest.mark.parametrize("shape", SHAPES)
def test_fp8_split_k_against_quantised_product(shape, two):
    m, n, p = shape
    A, B = inputs.row_col_scaled_f32(m, n, p, seed=m * 3 + n)
    fl = moa.MOA_FLAG_SPLIT_K(5) | (moa.MOA_FLAG_FP8_TWO_TERM if two else moa.MOA_FLAG_FP8_ONE_TERM)
    C = run(A, B, "fp8", fl)
    Q = O.fp8_gemm_2term(A, B) if two else O.fp8_gemm(A, B)
    assert O.rel_err(C, Q) <= 1e-4
    assert np.array_equal(C, run(A, B, "fp8", fl))


@pytest.mark.parametrize("path,flags", [("split_bf16", 0), ("fp8", moa.MOA_FLAG_FP8_ONE_TERM), ("fp8", moa.MOA_FLAG_FP8_TWO_TERM)])
def test_split_k_integer_exact_and_accumulate(path, flags):
    A, B = inputs.integer_valued(70, 3000, 90, seed=12, dtype=np.float32)
    C0 = (np.arange(70 * 90, dtype=np.float32).reshape(70, 90) % 11)
    R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
    fl = flags | moa.MOA_FLAG_SPLIT_K(9)
    assert np.array_equal(run(A, B, path, fl).astype(np.float64), R)
    assert np.array_equal(run(A, B, path, fl, accumulate=True, C0=C0).astype(np.float64),
                          R + C0.astype(np.float64))


def test_split_k_more_chunks_than_slabs():
    """n = 40 gives 3 slabs of 16: a request for 64 chunks runs 3."""
    A, B = inputs.normal_f32(50, 40, 60, seed=3)
    C = run(A, B, "split_bf16", moa.MOA_FLAG_SPLIT_K(64))
    assert O.rel_err(C, O.gemm_f64(A.astype(np.float64), B.astype(np.float64))) <= 1e-5


def test_grouped_split_k_member_equals_single_and_prepared_group_refuses():
    shapes = [(90, 4000, 70), (200, 300, 150), (64, 8000, 64)]
    ops = inputs.grouped_operands(shapes, seed=17)
    flags = [moa.MOA_FLAG_SPLIT_K(6), 0, moa.MOA_FLAG_SPLIT_K(12)]
    descs, outs, refs = [], [], []
    for (A, B), fl in zip(ops, flags):
        At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
        Ct = torch.empty((A.shape[0], B.shape[1]), device=DEV)
        Rt = torch.empty_like(Ct)
        moa.moa_gemm(At, Bt, Rt, path="split_bf16", flags=fl)
        descs.append(moa.make_desc(At, Bt, Ct, path="split_bf16", flags=fl))
        outs.append((At, Bt, Ct))
        refs.append(Rt)
    moa.moa_gemm_grouped(descs)
    torch.cuda.synchronize()
    for (_, _, Ct), Rt in zip(outs, refs):
        assert torch.equal(Ct, Rt)
    with pytest.raises(moa.MoaError) as ei:
        moa.moa_group_create(descs)
    assert ei.value.status == moa.MOA_ERR_UNSUPPORTED


@pytest.mark.parametrize("path,flags", [("split_bf16", 0), ("fp8", moa.MOA_FLAG_FP8_TWO_TERM)])
def test_planner_chosen_split_k(path, flags):
    """A skinny product with a long k walk is split by the planner itself: the
    same bits as asking for the planner's chunk count, the path's bar against
    the oracle, and a grouped launch runs it singly (alone = in the group)."""
    m, n, p = 96, 6000, 130
    A, B = inputs.normal_f32(m, n, p, seed=41)
    At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    C = torch.full((m, p), float("nan"), device=DEV)
    chunks = moa.moa_plan_query(moa.make_desc(At, Bt, C, path=path, flags=flags))["split_k"]
    assert chunks > 1
    auto = run(A, B, path, flags)
    assert np.array_equal(auto, run(A, B, path, flags | moa.MOA_FLAG_SPLIT_K(chunks)))
    whole = run(A, B, path, flags | moa.MOA_FLAG_SPLIT_K(1))
    if path == "split_bf16":
        R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
        assert O.rel_err(auto, R) <= 1e-5 and O.rel_err(whole, R) <= 1e-5
    else:
        Q = O.fp8_gemm_2term(A, B)
        assert O.rel_err(auto, Q) <= 1e-4 and O.rel_err(whole, Q) <= 1e-4
    small = inputs.normal_f32(70, 90, 50, seed=42)
    S = [torch.from_numpy(x).to(DEV) for x in small]
    Cs = torch.empty((70, 50), device=DEV)
    moa.moa_gemm_grouped([moa.make_desc(At, Bt, C, path=path, flags=flags),
                          moa.make_desc(S[0], S[1], Cs, path=path, flags=flags)])
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), auto)
