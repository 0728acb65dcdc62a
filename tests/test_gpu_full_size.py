"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

Row i of C depends only on row i of A (Eq. 3), so the oracle evaluated on A[rows]
against the whole of B is the exact reference for those rows of C; every check below
compares seeded sampled rows one by one.

* Square FP32 product N = 8192 with the benchmark's operands (N(0,1), seed N):
  split-BF16 with the planner's default block variant, the one the benchmark times,
  <= 1e-5 normwise against Eq. 3 in FP64 and <= sqrt(n) 2^-24 (FP32 accumulation only)
  against the exact three-term split product; ONF FP32 bitwise against the fma-ordered
  oracle; MFMA FP32 <= 1e-5.
* Precision workload m = 8192, n = 4096, p = 8192 (rows of A and columns of B scaled by
  10^U(-3,3), seed 3): split-BF16 and MFMA FP32 <= 1e-5 against Eq. 3; ONF FP32 bitwise;
  FP8 one- and two-term <= 1e-4 against the exact product of the quantised operands.
* N = 16384 split-BF16, the largest square size of the sweep.
* 256^3 FP64 (uniform [-1, 1), seed 0): ONF bitwise against the fma-ordered oracle and
  <= 1e-12 against Eq. 3.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_11148_amd import inputs, moa

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def sample_rows(m, count, seed):
    return np.sort(np.random.default_rng(seed).choice(m, size=count, replace=False))


def run(At, Bt, path, flags=0):
    Ct = torch.full((At.shape[0], Bt.shape[1]), float("nan"), dtype=At.dtype, device=DEV)
    moa.moa_gemm(At, Bt, Ct, path=path, flags=flags)
    torch.cuda.synchronize()
    return Ct


@pytest.fixture(scope="module")
def square8192():
    N = 8192
    A, B = inputs.normal_f32(N, N, N, seed=N)
    At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    yield A, B, At, Bt
    del At, Bt
    torch.cuda.empty_cache()


def test_square_8192_split_bf16_benchmark_plan(square8192):
    A, B, At, Bt = square8192
    C = torch.empty((8192, 8192), device=DEV)
    plan = moa.moa_plan_query(moa.make_desc(At, Bt, C, path="split_bf16"))
    assert (plan["tile_m"], plan["tile_n"], plan["workgroups"]) == (256, 256, 1024)
    Ct = run(At, Bt, "split_bf16")
    rows = sample_rows(8192, 32, seed=81)
    got = Ct[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    assert O.rel_err(got, O.gemm_rows_f64(A, B, rows)) <= 1e-5
    # against the exact three-term product only FP32 accumulation remains: n
    # independently rounded additions give a normwise error of about sqrt(n) u
    # (u = 2^-24), 5.4e-6 here; a dropped term would show as ~2^-8
    assert O.rel_err(got, O.split_bf16_gemm(A[rows], B)) <= np.sqrt(8192) * 2.0 ** -24
    assert np.all(np.isfinite(Ct.cpu().numpy()))          # every element written


def test_square_8192_onf_f32_bitwise(square8192):
    A, B, At, Bt = square8192
    Ct = run(At, Bt, "onf")
    rows = sample_rows(8192, 16, seed=82)
    got = Ct[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    assert np.array_equal(got, O.gemm_f32_fma(A[rows], B))


def test_square_8192_mfma_f32(square8192):
    A, B, At, Bt = square8192
    Ct = run(At, Bt, "mfma_f32")
    rows = sample_rows(8192, 32, seed=83)
    got = Ct[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    assert O.rel_err(got, O.gemm_rows_f64(A, B, rows)) <= 1e-5


@pytest.fixture(scope="module")
def precision_workload():
    A, B = inputs.row_col_scaled_f32(8192, 4096, 8192, seed=3)
    At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    yield A, B, At, Bt
    del At, Bt
    torch.cuda.empty_cache()


@pytest.mark.parametrize("path", ["split_bf16", "mfma_f32", "onf", "fp8", "fp8_two"])
def test_precision_workload_every_path(precision_workload, path):
    A, B, At, Bt = precision_workload
    flags = moa.MOA_FLAG_FP8_TWO_TERM if path == "fp8_two" else moa.MOA_FLAG_FP8_ONE_TERM if path == "fp8" else 0
    Ct = run(At, Bt, "fp8" if path == "fp8_two" else path, flags)
    rows = sample_rows(8192, 24, seed=84)
    got = Ct[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    if path == "onf":
        assert np.array_equal(got, O.gemm_f32_fma(A[rows], B))
    elif path == "fp8":
        assert O.rel_err(got, O.fp8_gemm(A[rows], B)) <= 1e-4
    elif path == "fp8_two":
        assert O.rel_err(got, O.fp8_gemm_2term(A[rows], B)) <= 1e-4
    else:
        assert O.rel_err(got, O.gemm_rows_f64(A, B, rows)) <= 1e-5


def test_square_16384_split_bf16():
    N = 16384
    A, B = inputs.normal_f32(N, N, N, seed=N)
    At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    Ct = run(At, Bt, "split_bf16")
    rows = sample_rows(N, 8, seed=85)
    got = Ct[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    del At, Bt, Ct
    torch.cuda.empty_cache()
    assert O.rel_err(got, O.gemm_rows_f64(A, B, rows)) <= 1e-5


def test_cube_256_f64_onf():
    A, B = inputs.uniform_f64(256, 256, 256, seed=0)
    At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    got = run(At, Bt, "onf").cpu().numpy()
    assert np.array_equal(got, O.gemm_f64_fma(A, B))
    assert O.rel_err(got, O.gemm_f64(A, B)) <= 1e-12


def test_square_8192_onf_f64_ring_bitwise():
    """The FP64 workload of the benchmark (8192^3, uniform[-1, 1), seed 8192) in
    its launch configuration (the direct-load ring kernel): sampled rows
    bitwise the fma-ordered oracle, every element written."""
    A, B = inputs.uniform_f64(8192, 8192, 8192, seed=8192)
    At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    Ct = torch.full((8192, 8192), float("nan"), dtype=torch.float64, device=DEV)
    d = moa.make_desc(At, Bt, Ct, path="onf")
    assert moa.moa_plan_query(d)["variant"] == 4
    moa.moa_gemm(At, Bt, Ct, path="onf")
    torch.cuda.synchronize()
    rows = sample_rows(8192, 12, seed=83)
    got = Ct[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    assert np.array_equal(got, O.gemm_f64_fma(A[rows], B))
    assert bool(torch.isfinite(Ct).all())
