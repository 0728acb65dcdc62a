"""The ipophp family on the GPU: Hadamard and Kronecker products bitwise equal
to the oracle's definitions (one rounded product per element; the accumulate
form adds it to C with a second rounding), and batched products as one grouped
launch (each member within its path's bar, bitwise equal to its single
launch)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_11148_amd import inputs, moa

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (64, 64), (257, 1001), (1024, 1023)])
def test_hadamard_bitwise(shape, dt):
    rng = np.random.default_rng(sum(shape))
    A, B, C0 = (rng.standard_normal(shape).astype(dt) for _ in range(3))
    At, Bt = dev(A), dev(B)
    Ct = torch.full(shape, float("nan"), dtype=At.dtype, device=DEV)
    moa.moa_hadamard(At, Bt, Ct)
    torch.cuda.synchronize()
    assert np.array_equal(Ct.cpu().numpy(), O.hadamard(A, B))
    Ct = dev(C0)
    moa.moa_hadamard(At, Bt, Ct, accumulate=True)
    torch.cuda.synchronize()
    assert np.array_equal(Ct.cpu().numpy(), O.hadamard(A, B, C0, accumulate=True))


def test_hadamard_in_place_and_unaligned():
    rng = np.random.default_rng(9)
    A, B = (rng.standard_normal(4099).astype(np.float32) for _ in range(2))
    At, Bt = dev(A), dev(B)
    moa.moa_hadamard(At.view(1, -1), Bt.view(1, -1), At.view(1, -1))       # C is A
    torch.cuda.synchronize()
    assert np.array_equal(At.cpu().numpy(), O.hadamard(A, B))
    # operands at a 4-byte offset: the scalar path
    X = dev(np.concatenate([[0.0], A]).astype(np.float32))
    Y = dev(np.concatenate([[0.0], B]).astype(np.float32))
    Z = torch.empty(4100, device=DEV)
    moa.moa_hadamard(X[1:].view(1, -1), Y[1:].view(1, -1), Z[1:].view(1, -1))
    torch.cuda.synchronize()
    assert np.array_equal(Z[1:].cpu().numpy(), O.hadamard(A, B))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shapes", [((1, 1), (1, 1)), ((2, 3), (5, 7)), ((7, 4), (3, 9)), ((16, 16), (33, 65))])
def test_kronecker_bitwise(shapes, dt):
    rng = np.random.default_rng(11)
    A = rng.standard_normal(shapes[0]).astype(dt)
    B = rng.standard_normal(shapes[1]).astype(dt)
    (m, n), (p, q) = shapes
    Ct = torch.full((m * p, n * q), float("nan"), dtype=dev(A).dtype, device=DEV)
    moa.moa_kronecker(dev(A), dev(B), Ct)
    torch.cuda.synchronize()
    R = O.kronecker(A, B)
    assert np.array_equal(Ct.cpu().numpy(), R)
    C0 = rng.standard_normal((m * p, n * q)).astype(dt)
    Ct = dev(C0)
    moa.moa_kronecker(dev(A), dev(B), Ct, accumulate=True)
    torch.cuda.synchronize()
    assert np.array_equal(Ct.cpu().numpy(), O.kronecker(A, B, C0, accumulate=True))


def test_kronecker_large_output():
    """64 x 64 (x) 128 x 128 -> 8192 x 8192 FP32 (the benchmark's size)."""
    rng = np.random.default_rng(12)
    A = rng.standard_normal((64, 64)).astype(np.float32)
    B = rng.standard_normal((128, 128)).astype(np.float32)
    Ct = torch.empty((8192, 8192), device=DEV)
    moa.moa_kronecker(dev(A), dev(B), Ct)
    torch.cuda.synchronize()
    assert np.array_equal(Ct.cpu().numpy(), O.kronecker(A, B))


@pytest.mark.parametrize("path", ["split_bf16", "onf"])
def test_batched_products(path):
    batch, m, n, p = 12, 130, 200, 90
    dt = np.float64 if path == "onf" else np.float32
    rng = np.random.default_rng(13)
    A = rng.standard_normal((batch, m, n)).astype(dt)
    B = rng.standard_normal((batch, n, p)).astype(dt)
    At, Bt = dev(A), dev(B)
    Ct = torch.full((batch, m, p), float("nan"), dtype=At.dtype, device=DEV)
    moa.moa_gemm_batched(At, Bt, Ct, path=path)
    torch.cuda.synchronize()
    got = Ct.cpu().numpy()
    for b in range(batch):
        single = torch.empty((m, p), dtype=At.dtype, device=DEV)
        moa.moa_gemm(At[b], Bt[b], single, path=path)
        torch.cuda.synchronize()
        assert np.array_equal(got[b], single.cpu().numpy())
    if path == "onf":
        assert all(np.array_equal(got[b], O.gemm_f64_fma(A[b], B[b])) for b in range(batch))
    else:
        assert O.rel_err(got, O.gemm_batched(A, B)) <= 1e-5
