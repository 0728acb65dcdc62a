"""moa_gemm_noalloc (scratch in the library's fixed per-GPU array) against
moa_gemm, through the C ABI.

Both entry points run the same plan and kernels, so the bar is bitwise
equality with moa_gemm's C; each result is also held to its path's bar
against Eq. 3 in FP64 (1e-5 for the FP32 matrix cores and split-BF16, 3e-2
for two-term scaled FP8, bitwise for ONF against the fma-ordered oracle).
Two calls run back to back on one stream, the second on a smaller product,
so the second reuses the array the first left behind.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_11148_amd import inputs, moa

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
BIG, SMALL = (700, 900, 500), (129, 200, 77)

CASES = [
    ("split_bf16", 0, 1e-5),
    ("fp8", 0, 3e-2),
    ("fp8", moa.MOA_FLAG_FP8_ONE_TERM, 5e-2),
    ("mfma_f32", 0, 1e-5),
    ("split_bf16", moa.MOA_FLAG_SPLIT_K(4), 1e-5),
    ("fp8", moa.MOA_FLAG_SPLIT_K(3), 3e-2),
]


def _operands(shape, seed):
    m, n, p = shape
    A, B = inputs.normal_f32(m, n, p, seed=seed)
    return A, B, torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)


@pytest.mark.parametrize("path,flags,bar", CASES)
@pytest.mark.parametrize("accumulate", [False, True])
def test_noalloc_equals_moa_gemm_two_calls(path, flags, bar, accumulate):
    print(f"noalloc {path} flags={flags:#x} accumulate={accumulate}", flush=True)
    runs = []
    for shape, seed in ((BIG, 11), (SMALL, 12)):
        A, B, At, Bt = _operands(shape, seed)
        m, _, p = shape
        C0 = np.random.default_rng(seed + 100).standard_normal((m, p)).astype(np.float32)
        ref = torch.from_numpy(C0).to(DEV) if accumulate else torch.full((m, p), float("nan"), device=DEV)
        out = ref.clone()
        runs.append((A, B, C0, At, Bt, ref, out))
    torch.cuda.synchronize()
    for A, B, C0, At, Bt, ref, out in runs:          # back to back on one stream, no sync between
        moa.moa_gemm_noalloc(At, Bt, out, path=path, accumulate=accumulate, flags=flags)
    for A, B, C0, At, Bt, ref, out in runs:
        moa.moa_gemm(At, Bt, ref, path=path, accumulate=accumulate, flags=flags)
    torch.cuda.synchronize()
    for A, B, C0, At, Bt, ref, out in runs:
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(got, want), f"{path}: noalloc differs from moa_gemm at {A.shape[0]}x{B.shape[1]}"
        R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
        if accumulate:
            R = R + C0.astype(np.float64)
        assert O.rel_err(got, R) <= bar


def test_noalloc_onf_bitwise():
    A, B, At, Bt = _operands(SMALL, 13)
    C = torch.full((SMALL[0], SMALL[2]), float("nan"), device=DEV)
    moa.moa_gemm_noalloc(At, Bt, C, path="onf")
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), O.gemm_f32_fma(A, B))


def test_noalloc_refuses_products_beyond_the_array():
    m = n = p = 4096                     # split-BF16 records of A and B: 128 MiB
    d = moa.moa_gemm_desc(m=m, n=n, p=p, dtype=moa.MOA_F32, path=moa.MOA_PATH_SPLIT_BF16, A=16, B=16,
                          C=1 << 40, accumulate=0, flags=0)
    assert moa.moa_plan_query(d)["workspace_bytes"] > moa.MOA_NOALLOC_SCRATCH_BYTES
    At = torch.zeros((m, n), device=DEV)
    Bt = torch.zeros((n, p), device=DEV)
    C = torch.full((m, p), 7.0, device=DEV)
    with pytest.raises(moa.MoaError) as ei:
        moa.moa_gemm_noalloc(At, Bt, C, path="split_bf16")
    assert ei.value.status == moa.MOA_ERR_NOMEM
    torch.cuda.synchronize()
    assert bool((C == 7.0).all())          # nothing launched
    # the array is still usable afterwards
    test_noalloc_onf_bitwise()
    A, B, At, Bt = _operands(SMALL, 14)
    C1 = torch.empty((SMALL[0], SMALL[2]), device=DEV)
    C2 = torch.empty_like(C1)
    moa.moa_gemm_noalloc(At, Bt, C1, path="split_bf16")
    moa.moa_gemm(At, Bt, C2, path="split_bf16")
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
