"""Writes stay inside C; inputs stay untouched.

Every operand lives inside a larger device buffer whose margins (4 KiB of
elements on each side) hold a sentinel bit pattern; A and B are filled with
data, C with NaN. After each launch -- every path, every block variant, split-k,
column-major operands, grouped launches, Hadamard and Kronecker products, on
ragged shapes that leave partial tiles in every direction -- the margins and
the inputs must be bitwise unchanged and every element of C written (finite).
"""
import itertools

import pytest
import torch

from paper_2306_11148_amd import moa

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GUARD = 1024                               # elements of margin on each side
SENTINEL = {torch.float32: 0x7FBADBAD, torch.float64: 0x7FF4BADBADBADBAD}
INT = {torch.float32: torch.int32, torch.float64: torch.int64}


class Guarded:
    """A rows x cols matrix inside a guarded buffer (row- or column-major)."""

    def __init__(self, rows, cols, dtype, fill=None, col=False, seed=0):
        self.buf = torch.empty(rows * cols + 2 * GUARD, dtype=dtype, device=DEV)
        self.buf.view(INT[dtype]).fill_(SENTINEL[dtype])
        body = self.buf[GUARD:GUARD + rows * cols]
        self.t = body.view(cols, rows).t() if col else body.view(rows, cols)
        if fill == "nan":
            self.t.fill_(float("nan"))
        elif fill is not None:
            g = torch.Generator(device=DEV).manual_seed(seed)
            self.t.copy_(torch.randn((rows, cols), generator=g, device=DEV, dtype=dtype))
        self.snapshot = self.buf.clone()

    def margins_intact(self):
        head = torch.equal(self.buf[:GUARD].view(INT[self.buf.dtype]),
                           self.snapshot[:GUARD].view(INT[self.buf.dtype]))
        tail = torch.equal(self.buf[-GUARD:].view(INT[self.buf.dtype]),
                           self.snapshot[-GUARD:].view(INT[self.buf.dtype]))
        return head and tail

    def unchanged(self):
        return torch.equal(self.buf.view(INT[self.buf.dtype]), self.snapshot.view(INT[self.buf.dtype]))


def check(A, B, C):
    torch.cuda.synchronize()
    assert A.unchanged() and B.unchanged(), "an input was written"
    assert C.margins_intact(), "a write landed outside C"
    assert bool(torch.isfinite(C.t).all()), "an element of C was not written"


SHAPES = [(130, 77, 258), (1, 33, 1), (257, 1000, 129), (64, 16, 64)]


def variant_count(path, flags, dtype):
    d = moa.moa_gemm_desc(m=300, n=300, p=300, dtype=moa.MOA_F64 if dtype == torch.float64 else moa.MOA_F32,
                          path=moa.PATHS[path], A=16, B=16, C=1 << 20, accumulate=0, flags=flags)
    v = 0
    while True:
        d.flags = flags | moa.MOA_FLAG_VARIANT(v)
        try:
            moa.moa_plan_query(d)
        except moa.MoaError:
            return v
        v += 1


CASES = [("onf", 0, torch.float64), ("onf", 0, torch.float32), ("mfma_f32", 0, torch.float32),
         ("split_bf16", 0, torch.float32), ("fp8", moa.MOA_FLAG_FP8_ONE_TERM, torch.float32),
         ("fp8", moa.MOA_FLAG_FP8_TWO_TERM, torch.float32)]


@pytest.mark.parametrize("path,flags,dtype", CASES)
@pytest.mark.parametrize("shape", SHAPES)
def test_every_variant_writes_only_c(path, flags, dtype, shape):
    m, n, p = shape
    for v in range(variant_count(path, flags, dtype)):
        A = Guarded(m, n, dtype, fill="data", seed=1)
        B = Guarded(n, p, dtype, fill="data", seed=2)
        C = Guarded(m, p, dtype, fill="nan")
        moa.moa_gemm(A.t, B.t, C.t, path=path, flags=flags | moa.MOA_FLAG_VARIANT(v))
        check(A, B, C)


@pytest.mark.parametrize("path,flags", [("split_bf16", 0), ("fp8", moa.MOA_FLAG_FP8_ONE_TERM), ("fp8", moa.MOA_FLAG_FP8_TWO_TERM)])
@pytest.mark.parametrize("shape", SHAPES)
def test_split_k_writes_only_c(path, flags, shape):
    m, n, p = shape
    A = Guarded(m, n, torch.float32, fill="data", seed=3)
    B = Guarded(n, p, torch.float32, fill="data", seed=4)
    C = Guarded(m, p, torch.float32, fill="nan")
    moa.moa_gemm(A.t, B.t, C.t, path=path, flags=flags | moa.MOA_FLAG_SPLIT_K(5))
    check(A, B, C)


@pytest.mark.parametrize("combo", list(itertools.product([False, True], repeat=3)))
@pytest.mark.parametrize("path", ["split_bf16", "fp8", "onf", "mfma_f32"])
def test_column_major_operands_write_only_c(path, combo):
    m, n, p = 130, 300, 77
    a_col, b_col, c_col = combo
    A = Guarded(m, n, torch.float32, fill="data", col=a_col, seed=5)
    B = Guarded(n, p, torch.float32, fill="data", col=b_col, seed=6)
    C = Guarded(m, p, torch.float32, fill="nan", col=c_col)
    moa.moa_gemm(A.t, B.t, C.t, path=path)
    check(A, B, C)


def test_grouped_members_write_only_their_c():
    shapes = [(130, 77, 258), (1, 33, 1), (257, 1000, 129), (64, 16, 64), (300, 500, 3)]
    paths = [("split_bf16", 0), ("fp8", moa.MOA_FLAG_FP8_ONE_TERM), ("fp8", moa.MOA_FLAG_FP8_TWO_TERM), ("onf", 0), ("mfma_f32", 0)]
    members, descs = [], []
    for k, (m, n, p) in enumerate(shapes):
        for path, flags in paths:
            A = Guarded(m, n, torch.float32, fill="data", seed=10 + k)
            B = Guarded(n, p, torch.float32, fill="data", seed=20 + k)
            C = Guarded(m, p, torch.float32, fill="nan")
            members.append((A, B, C))
            descs.append(moa.make_desc(A.t, B.t, C.t, path=path, flags=flags))
    moa.moa_gemm_grouped(descs)
    for A, B, C in members:
        check(A, B, C)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_hadamard_and_kronecker_write_only_c(dtype):
    A = Guarded(130, 77, dtype, fill="data", seed=7)
    B = Guarded(130, 77, dtype, fill="data", seed=8)
    C = Guarded(130, 77, dtype, fill="nan")
    moa.moa_hadamard(A.t, B.t, C.t)
    check(A, B, C)
    A = Guarded(13, 7, dtype, fill="data", seed=9)
    B = Guarded(11, 29, dtype, fill="data", seed=10)
    C = Guarded(13 * 11, 7 * 29, dtype, fill="nan")
    moa.moa_kronecker(A.t, B.t, C.t)
    check(A, B, C)
