"""The longest k walks the ring paths accept (n = 16 * 131071 on split-BF16,
64 * 131071 on FP8: the last slab's records sit at the top of the 32-bit
offset range of a row tile), on a thin product m = 3, p = 5.

Integer-valued operands in [-8, 8] are exact in BF16 and, after the power-of-two
row and column scaling, in E4M3, and every partial sum stays an integer far
below 2^24, so each path must reproduce Eq. 3 exactly: a wrong offset in any
slab (a dropped, repeated or misplaced record) changes the result.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_11148_amd import inputs, moa

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("path,flags,k", [
    ("split_bf16", 0, 16),
    ("split_bf16", moa.MOA_FLAG_SPLIT_K(7), 16),
    ("fp8", moa.MOA_FLAG_FP8_ONE_TERM, 64),
    ("fp8", moa.MOA_FLAG_FP8_TWO_TERM, 64),
])
def test_longest_k_walk_exact(path, flags, k):
    n = k * 131071
    A, B = inputs.integer_valued(3, n, 5, seed=k + flags % 97, dtype=np.float32)
    R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
    assert np.abs(R).max() < 2 ** 24
    At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    Ct = torch.full((3, 5), float("nan"), device=DEV)
    moa.moa_gemm(At, Bt, Ct, path=path, flags=flags)
    torch.cuda.synchronize()
    assert np.array_equal(Ct.cpu().numpy().astype(np.float64), R)
