"""Host-side checks of the C ABI (no GPU needed, nothing is launched).

* libmoa.so loads and exports every function include/moa.h declares.
* The block-size rule of section "Technical Details" reproduces the paper's
  numbers (tests/golden/static_rule_paper.json) and agrees with the oracle's
  statement of the same rule.
* Argument errors (Eq. 1-2 shape and index rules) come back synchronously.
* Planning (the dimension lift) is a pure host function.
"""
import ctypes
import json
import os
import re

import pytest

from oracle import oracle as O
from paper_2306_11148_amd import inputs, moa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "moa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(moa_[a-z0-9_]+)\s*\(", text)) - {"moa_gemm_desc"})


def test_library_exports_every_declared_function():
    L = moa.lib()
    names = header_functions()
    assert "moa_gemm" in names and "moa_serve_submit" in names
    for name in names:
        assert hasattr(L, name), f"{name} declared in include/moa.h but not exported"
    assert sorted(moa.EXPORTS) == names


def test_static_rule_matches_paper_and_oracle():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "static_rule_paper.json")))
    for c in g["cases"]:
        assert moa.moa_static_block_components(c["budget_bytes"], c["elem_bytes"], c["nblocks"]) \
            == c["components"]
    for budget in (0, 1, 23, 24, 25, 4096, 32768, 98304, 131072, 163840, 10**9):
        for es in (1, 2, 4, 8):
            for nb in (1, 2, 3):
                assert moa.moa_static_block_components(budget, es, nb) == \
                    O.static_block_components(budget, es, nb)
    assert moa.moa_static_block_components(-1, 8, 3) == 0
    assert moa.moa_static_block_components(32768, 0, 3) == 0


def _desc(m, n, p, dtype=moa.MOA_F32, path=moa.MOA_PATH_AUTO, A=0x1000, B=0x100000000,
          C=0x200000000, acc=0, flags=0):
    return moa.moa_gemm_desc(m, n, p, dtype, path, A, B, C, acc, flags)


def test_plan_static_components_and_shapes():
    q = moa.moa_plan_query(_desc(256, 256, 256, moa.MOA_F64))
    assert q["path"] == moa.MOA_PATH_ONF
    assert q["static_components"] == 1024            # 32 x 32 doubles in a 32 KB L1
    q0 = moa.moa_plan_query(_desc(256, 256, 256, moa.MOA_F64, flags=moa.MOA_FLAG_VARIANT(0)))
    assert q0["tile_m"] * q0["tile_n"] == 1024       # the static block itself
    q32 = moa.moa_plan_query(_desc(256, 256, 256, moa.MOA_F32, moa.MOA_PATH_ONF,
                                   flags=moa.MOA_FLAG_VARIANT(0)))
    assert q32["static_components"] == 2048 and q32["tile_m"] * q32["tile_n"] == 2048
    big = moa.moa_plan_query(_desc(8192, 8192, 8192))
    assert big["path"] == moa.MOA_PATH_SPLIT_BF16
    assert big["workgroups"] >= 256
    f8 = moa.moa_plan_query(_desc(100, 200, 300, path=moa.MOA_PATH_FP8_SCALED))
    assert f8["workspace_bytes"] >= 100 * 200 + 200 * 300


def test_fp8_plan_variants():
    """FP8 block variants: 64-code slabs, LDS ring of three slabs of records
    (two record arrays per operand for the two-term form), largest block with
    a workgroup per CU by default."""
    F8 = moa.MOA_PATH_FP8_SCALED
    TWO = moa.MOA_FLAG_FP8_TWO_TERM
    ONE = moa.MOA_FLAG_FP8_ONE_TERM
    one = [moa.moa_plan_query(_desc(1000, 300, 1000, path=F8, flags=ONE | moa.MOA_FLAG_VARIANT(v))) for v in range(2)]
    assert [(q["tile_m"], q["tile_n"], q["tile_k"]) for q in one] == [(128, 128, 64), (256, 256, 64)]
    assert [q["lds_bytes"] for q in one] == [3 * 256 * 64, 3 * 512 * 64]
    two = [moa.moa_plan_query(_desc(1000, 300, 1000, path=F8, flags=TWO | moa.MOA_FLAG_VARIANT(v)))
           for v in range(2)]
    assert [q["threads"] for q in two] == [256, 512]
    assert all(q["lds_bytes"] == 3 * 2 * 256 * 64 for q in two)
    assert call(_desc(8, 8, 8, path=F8, flags=moa.MOA_FLAG_VARIANT(9))) == moa.MOA_ERR_INVALID
    # records: padded rows x ceil(n / 64) x 64 bytes per operand (twice for two terms)
    q1 = moa.moa_plan_query(_desc(100, 200, 300, path=F8, flags=ONE))
    q2 = moa.moa_plan_query(_desc(100, 200, 300, path=F8, flags=TWO))
    rec = (112 + 304) * 4 * 64
    assert rec <= q1["workspace_bytes"] < rec + 8 * 1024
    assert 2 * rec <= q2["workspace_bytes"] < 2 * rec + 8 * 1024
    big = moa.moa_plan_query(_desc(8192, 8192, 8192, path=F8, flags=ONE))
    assert big["tile_m"] == 256 and big["workgroups"] == 1024
    # two terms are the default; both flags together are refused
    assert moa.moa_plan_query(_desc(100, 200, 300, path=F8)) == q2
    assert call(_desc(8, 8, 8, path=F8, flags=ONE | TWO)) == moa.MOA_ERR_INVALID


def test_split_default_block_rule():
    """256x256 once every CU gets a block, 128x128 below; rectangular blocks
    (orientation by the longer side) when the last round of 256x256 blocks
    would be less than 40% full."""
    S16 = moa.MOA_PATH_SPLIT_BF16
    shape = lambda m, p: (lambda q: (q["variant"], q["tile_m"], q["tile_n"]))(
        moa.moa_plan_query(_desc(m, 1024, p, path=S16)))
    assert shape(3072, 3072) == (0, 128, 128)          # 144 big blocks
    assert shape(4096, 4096) == (1, 256, 256)          # one whole round
    assert shape(5120, 5120) == (1, 256, 256)          # 1.56 rounds
    assert shape(6144, 6144) == (3, 128, 256)          # 2.25 rounds
    assert shape(6400, 6144) == (2, 256, 128)          # 600 blocks, m > p
    assert shape(8192, 8192) == (1, 256, 256)          # four whole rounds


def test_fp8_one_term_default_shortens_the_last_round():
    F8 = moa.MOA_PATH_FP8_SCALED
    ONE = moa.MOA_FLAG_FP8_ONE_TERM
    assert moa.moa_plan_query(_desc(8192, 4096, 8192, path=F8, flags=ONE))["tile_m"] == 256    # 4 whole rounds
    assert moa.moa_plan_query(_desc(6144, 6144, 6144, path=F8, flags=ONE))["variant"] == 0     # 2.25 rounds


def test_split_k_plan():
    """Split-k: chunks clamped so none is empty, partials in the workspace,
    one workgroup per (block, chunk), first block variant; ring paths only."""
    S16 = moa.MOA_PATH_SPLIT_BF16
    base = moa.moa_plan_query(_desc(100, 20000, 100, path=S16, flags=moa.MOA_FLAG_SPLIT_K(1)))
    q = moa.moa_plan_query(_desc(100, 20000, 100, path=S16, flags=moa.MOA_FLAG_SPLIT_K(8)))
    assert base["split_k"] == 1 and q["split_k"] == 8
    assert q["workgroups"] == 8 * base["workgroups"] and q["tile_m"] == 128
    assert q["workspace_bytes"] >= base["workspace_bytes"] + 8 * 100 * 100 * 4
    # n = 40 -> 3 slabs of 16: 8 chunks clamp to 3
    assert moa.moa_plan_query(_desc(64, 40, 64, path=S16, flags=moa.MOA_FLAG_SPLIT_K(8)))["split_k"] == 3
    # 10 slabs in 6 chunks -> chunks of 2 -> 5 chunks
    assert moa.moa_plan_query(_desc(64, 160, 64, path=S16, flags=moa.MOA_FLAG_SPLIT_K(6)))["split_k"] == 5
    f8 = moa.moa_plan_query(_desc(64, 640, 64, path=moa.MOA_PATH_FP8_SCALED,
                                  flags=moa.MOA_FLAG_FP8_TWO_TERM | moa.MOA_FLAG_SPLIT_K(4)))
    assert f8["split_k"] == 4 and f8["tile_k"] == 64          # 10 slabs of 64 -> chunks of 3 -> 4
    assert call(_desc(8, 8, 8, moa.MOA_F32, moa.MOA_PATH_ONF, flags=moa.MOA_FLAG_SPLIT_K(2))) == \
        moa.MOA_ERR_UNSUPPORTED
    assert call(_desc(8, 8, 8, flags=1 << 28)) == moa.MOA_ERR_INVALID


def test_onf_f64_ring_plan():
    """FP64 products with every CU given a 128 x 128 block run the direct-load
    ring kernel (variant 4) when their operands are row-major and their
    offsets fit; the others stay on the register-staged blocks."""
    F64, ONF = moa.MOA_F64, moa.MOA_PATH_ONF
    q = lambda m, n, p, fl=0: moa.moa_plan_query(_desc(m, n, p, F64, ONF, flags=fl))  # noqa: E731
    big = q(8192, 8192, 8192)
    assert big["variant"] == 4 and (big["tile_m"], big["tile_n"], big["tile_k"]) == (128, 128, 8)
    assert (big["lane_m"], big["lane_n"]) == (8, 8) and big["lds_bytes"] == 4 * 16384
    assert q(2048, 2048, 2048)["variant"] == 4                   # 256 blocks
    assert q(2048, 2048, 1920)["variant"] != 4                   # 240 blocks
    assert q(256, 256, 256)["variant"] == 0                      # the static rule's 32 x 32 block
    allcol = moa.MOA_FLAG_A_COL | moa.MOA_FLAG_B_COL | moa.MOA_FLAG_C_COL
    assert q(8192, 8192, 8192, allcol)["variant"] == 4          # C^T = B^T A^T is all row-major
    assert q(8192, 8192, 8192, moa.MOA_FLAG_A_COL)["variant"] == 2
    assert q(4096, 2100000, 4096)["variant"] == 2                # A's offsets would not fit
    with pytest.raises(moa.MoaError) as ei:
        q(256, 256, 256, moa.MOA_FLAG_VARIANT(4) | moa.MOA_FLAG_B_COL)
    assert ei.value.status == moa.MOA_ERR_UNSUPPORTED
    assert q(256, 256, 256, moa.MOA_FLAG_VARIANT(4))["variant"] == 4
    with pytest.raises(moa.MoaError):
        q(256, 256, 256, moa.MOA_FLAG_VARIANT(5))


def test_onf_f32_ring_plan():
    """FP32 products likewise: the direct-load ring kernel (variant 4, 16-k
    slabs, 128 x 128 blocks of 8 x 8 per lane, three-stage ring) once every
    CU gets a block and the operands are row-major; else the largest
    register-staged block that still gives every CU one."""
    F32, ONF = moa.MOA_F32, moa.MOA_PATH_ONF
    q = lambda m, n, p, fl=0: moa.moa_plan_query(_desc(m, n, p, F32, ONF, flags=fl))  # noqa: E731
    big = q(8192, 8192, 8192)
    assert big["variant"] == 4 and (big["tile_m"], big["tile_n"], big["tile_k"]) == (128, 128, 16)
    assert (big["lane_m"], big["lane_n"]) == (8, 8) and big["lds_bytes"] == 3 * 16384
    assert q(2048, 2048, 2048)["variant"] == 4                   # 256 blocks
    assert q(2048, 2048, 1920)["variant"] == 2                   # 240 blocks of 128 x 128: 64 x 128
    assert q(8192, 8192, 8192, moa.MOA_FLAG_A_COL)["variant"] == 3
    assert q(4096, 4200000, 4096)["variant"] == 3                # A's offsets would not fit
    with pytest.raises(moa.MoaError) as ei:
        q(256, 256, 256, moa.MOA_FLAG_VARIANT(4) | moa.MOA_FLAG_A_COL)
    assert ei.value.status == moa.MOA_ERR_UNSUPPORTED


def test_split_k_chosen_by_the_planner():
    """Without MOA_FLAG_SPLIT_K the planner splits products of at most 64
    blocks of 128 x 128 with n >= 4096 into about 512 workgroups of at least
    512 k each; MOA_FLAG_SPLIT_K(1) keeps them whole."""
    S16, F8 = moa.MOA_PATH_SPLIT_BF16, moa.MOA_PATH_FP8_SCALED
    q = lambda m, n, p, path=S16, fl=0: moa.moa_plan_query(_desc(m, n, p, path=path, flags=fl))  # noqa: E731
    assert q(256, 65536, 256)["split_k"] == 128                  # 4 blocks: 512 / 4, n / 512 = 128
    assert q(512, 32768, 512)["split_k"] == 32                   # 16 blocks
    assert q(1024, 16384, 1024)["split_k"] == 8                  # 64 blocks
    assert q(1024, 16384, 1024)["workgroups"] == 512
    assert q(100, 20000, 100)["split_k"] == 38                   # 39 asked: 1250 slabs in chunks of 33
    assert q(128, 4096, 128)["split_k"] == 8                     # capped by n / 512
    assert q(1152, 16384, 1024)["split_k"] == 1                  # 72 blocks: enough to spread
    assert q(256, 4095, 256)["split_k"] == 1                     # short k walk
    assert q(256, 65536, 256, fl=moa.MOA_FLAG_SPLIT_K(1))["split_k"] == 1
    assert q(256, 65536, 256, fl=moa.MOA_FLAG_SPLIT_K(3))["split_k"] == 3
    assert q(256, 65536, 256, path=F8)["split_k"] == 128         # FP8: the same rule (its slabs are 64 k)
    assert q(256, 65536, 256, path=moa.MOA_PATH_ONF)["split_k"] == 1
    assert q(256, 65536, 256, path=moa.MOA_PATH_MFMA_F32)["split_k"] == 1


def test_size_limits_at_the_boundary():
    """The record offsets inside one 16-row tile are 32-bit: n may reach
    16 * 131071 on split-BF16 (16 k per record) and 64 * 131071 on FP8 (64 k
    per record); one more is refused with MOA_ERR_SHAPE, before any launch."""
    cases = [(moa.MOA_PATH_SPLIT_BF16, 0, 16), (moa.MOA_PATH_FP8_SCALED, moa.MOA_FLAG_FP8_ONE_TERM, 64),
             (moa.MOA_PATH_FP8_SCALED, moa.MOA_FLAG_FP8_TWO_TERM, 64)]
    for path, flags, k in cases:
        q = moa.moa_plan_query(_desc(3, k * 131071, 5, path=path, flags=flags))
        assert q["tile_k"] == k and q["workspace_bytes"] > 0
        with pytest.raises(moa.MoaError) as ei:
            moa.moa_plan_query(_desc(3, k * 131071 + 1, 5, path=path, flags=flags))
        assert ei.value.status == moa.MOA_ERR_SHAPE
        assert call(_desc(3, k * 131071 + 1, 5, path=path, flags=flags)) == moa.MOA_ERR_SHAPE
    # ONF: at most 65535 row blocks
    tm = moa.moa_plan_query(_desc(8, 1, 1, moa.MOA_F32, moa.MOA_PATH_ONF, flags=moa.MOA_FLAG_VARIANT(0)))["tile_m"]
    moa.moa_plan_query(_desc(65535 * tm, 1, 1, moa.MOA_F32, moa.MOA_PATH_ONF, flags=moa.MOA_FLAG_VARIANT(0)))
    assert call(_desc(65535 * tm + 1, 1, 1, moa.MOA_F32, moa.MOA_PATH_ONF,
                      flags=moa.MOA_FLAG_VARIANT(0))) == moa.MOA_ERR_SHAPE


def test_mfma_f32_plan_variants():
    """FP32 matrix cores: record ring (128x128 / 256x256, scratch for the
    records) by default, the register-staged kernel (no scratch) as variant 2."""
    M = moa.MOA_PATH_MFMA_F32
    big = moa.moa_plan_query(_desc(8192, 8192, 8192, path=M))
    assert (big["variant"], big["tile_m"], big["tile_n"]) == (1, 256, 256)
    assert big["workspace_bytes"] == 4 * (8192 + 8192) * 8192
    small = moa.moa_plan_query(_desc(1000, 300, 1000, path=M))
    assert (small["variant"], small["tile_m"]) == (0, 128)
    staged = moa.moa_plan_query(_desc(8192, 8192, 8192, path=M, flags=moa.MOA_FLAG_VARIANT(2)))
    assert staged["workspace_bytes"] == 0 and staged["tile_k"] == 32
    assert call(_desc(8, 8, 8, path=M, flags=moa.MOA_FLAG_VARIANT(5))) == moa.MOA_ERR_INVALID
    tail = moa.moa_plan_query(_desc(6144, 1024, 6144, path=M))   # 576 blocks: 2.25 rounds
    assert (tail["variant"], tail["tile_m"], tail["tile_n"]) == (4, 128, 256)
    # the record ring's offsets bound n; the staged kernel has no such limit
    assert call(_desc(3, 16 * 131071 + 1, 5, path=M)) == moa.MOA_ERR_SHAPE
    moa.moa_plan_query(_desc(3, 16 * 131071 + 1, 5, path=M, flags=moa.MOA_FLAG_VARIANT(2)))


def test_layout_flags():
    """gamma_col operands: any combination on every path except the
    register-staged FP32 variant (row-major only); make_desc reads the layout
    from the strides."""
    import torch
    F32 = moa.MOA_F32
    allcol = moa.MOA_FLAG_A_COL | moa.MOA_FLAG_B_COL | moa.MOA_FLAG_C_COL
    for f in range(8):
        for path in (moa.MOA_PATH_ONF, moa.MOA_PATH_MFMA_F32):
            assert moa.moa_plan_query(_desc(8, 8, 8, F32, path, flags=f << 24))["path"] == path
        assert moa.moa_plan_query(_desc(8, 8, 8, moa.MOA_F64, moa.MOA_PATH_ONF, flags=f << 24))["path"] == 1
    staged = moa.MOA_FLAG_VARIANT(2)
    assert moa.moa_plan_query(_desc(8, 8, 8, F32, moa.MOA_PATH_MFMA_F32, flags=staged))["workspace_bytes"] == 0
    # all-column: C^T = B^T A^T is all row-major, so the staged kernel serves it
    assert moa.moa_plan_query(_desc(8, 8, 8, F32, moa.MOA_PATH_MFMA_F32, flags=staged | allcol))["variant"] == 2
    for f in (moa.MOA_FLAG_A_COL, moa.MOA_FLAG_B_COL, moa.MOA_FLAG_C_COL):
        with pytest.raises(moa.MoaError) as ei:
            moa.moa_plan_query(_desc(8, 8, 8, F32, moa.MOA_PATH_MFMA_F32, flags=staged | f))
        assert ei.value.status == moa.MOA_ERR_UNSUPPORTED
        assert call(_desc(8, 8, 8, F32, moa.MOA_PATH_MFMA_F32, flags=staged | f)) == moa.MOA_ERR_UNSUPPORTED
    for f in range(8):
        q = moa.moa_plan_query(_desc(100, 300, 2000, F32, moa.MOA_PATH_SPLIT_BF16, flags=f << 24))
        assert q["workgroups"] == 16
    A = torch.zeros(30, 20).t()                   # logical 20 x 30, column-major
    B = torch.zeros(30, 40)
    C = torch.zeros(20, 80)[:, ::2]               # every other column: neither layout
    d = moa.make_desc(A, B, torch.zeros(40, 20).t())
    assert (d.m, d.n, d.p) == (20, 30, 40)
    assert d.flags == moa.MOA_FLAG_A_COL | moa.MOA_FLAG_C_COL
    with pytest.raises(ValueError):
        moa.make_desc(A, B, C)


def test_ipophp_argument_errors_are_synchronous():
    L = moa.lib()
    F32, F64 = moa.MOA_F32, moa.MOA_F64
    assert L.moa_hadamard(-1, 2, F32, 0x1000, 0x2000, 0x3000, 0, None) == moa.MOA_ERR_SHAPE
    assert L.moa_hadamard(2, 2, 7, 0x1000, 0x2000, 0x3000, 0, None) == moa.MOA_ERR_INVALID
    assert L.moa_hadamard(2, 2, F32, None, 0x2000, 0x3000, 0, None) == moa.MOA_ERR_INVALID
    assert L.moa_hadamard(2, 2, F64, 0x1004, 0x2000, 0x3000, 0, None) == moa.MOA_ERR_INVALID    # misaligned
    assert L.moa_hadamard(4, 4, F32, 0x1000, 0x2000, 0x1000 + 8, 0, None) == moa.MOA_ERR_INVALID  # shifted C
    assert L.moa_hadamard(0, 5, F32, None, None, None, 0, None) == moa.MOA_OK                  # empty: no-op
    assert L.moa_kronecker(2, 1 << 16, 2, 1 << 16, F32, 0x1000, 0x2000, 0x3000, 0, None) == moa.MOA_ERR_SHAPE
    assert L.moa_kronecker(2, 2, 2, 2, F32, 0x1000, 0x2000, 0x1000, 0, None) == moa.MOA_ERR_INVALID  # C on A
    assert L.moa_kronecker(0, 3, 4, 5, F32, None, None, None, 0, None) == moa.MOA_OK
    d = _desc(4, 4, 4)
    assert L.moa_gemm_batched(ctypes.byref(d), -1, 16, 16, 16, None) == moa.MOA_ERR_INVALID
    assert L.moa_gemm_batched(ctypes.byref(d), 0, 16, 16, 16, None) == moa.MOA_OK
    # members' C overlap each other (stride smaller than m p)
    assert L.moa_gemm_batched(ctypes.byref(d), 3, 16, 16, 8, None) == moa.MOA_ERR_INVALID


def call(d):
    return moa.lib().moa_gemm(ctypes.byref(d), None)


def test_argument_errors_are_synchronous():
    L = moa.lib()
    assert L.moa_gemm(None, None) == moa.MOA_ERR_INVALID
    assert call(_desc(-1, 2, 3)) == moa.MOA_ERR_SHAPE
    assert call(_desc(2, 2, 2, dtype=7)) == moa.MOA_ERR_INVALID
    assert call(_desc(2, 2, 2, path=9)) == moa.MOA_ERR_INVALID
    assert call(_desc(2, 2, 2, flags=0x80)) == moa.MOA_ERR_INVALID
    assert call(_desc(2, 2, 2, moa.MOA_F64, moa.MOA_PATH_SPLIT_BF16)) == moa.MOA_ERR_UNSUPPORTED
    assert "ONF" in moa.moa_last_error()
    assert call(_desc(2, 2, 2, A=0)) == moa.MOA_ERR_INVALID
    # C overlapping A (the paper's program reads C while it writes it)
    assert call(_desc(4, 4, 4, A=0x1000, C=0x1000 + 16)) == moa.MOA_ERR_INVALID
    assert call(_desc(2**40, 2**40, 2)) == moa.MOA_ERR_SHAPE
    assert call(_desc(2, 2, 2, A=0x1002)) == moa.MOA_ERR_INVALID        # misaligned
    assert call(_desc(2, 2, 2, flags=moa.MOA_FLAG_VARIANT(40))) == moa.MOA_ERR_INVALID
    # empty outputs are a successful no-op and never touch the device
    assert call(_desc(0, 5, 7, A=0, C=0)) == moa.MOA_OK
    assert call(_desc(5, 7, 0, B=0, C=0)) == moa.MOA_OK
    assert L.moa_gemm_grouped(None, -1, None) == moa.MOA_ERR_INVALID
    assert L.moa_gemm_grouped(None, 1, None) == moa.MOA_ERR_INVALID
    assert L.moa_gemm_grouped(None, 0, None) == moa.MOA_OK


def test_status_strings():
    for code, name in [(0, "MOA_OK"), (1, "MOA_ERR_INVALID"), (2, "MOA_ERR_SHAPE"),
                       (3, "MOA_ERR_UNSUPPORTED"), (4, "MOA_ERR_NOMEM"), (5, "MOA_ERR_DEVICE"),
                       (6, "MOA_NOT_READY")]:
        assert moa.status_name(code) == name
    assert moa.status_name(99) == "MOA_UNKNOWN_STATUS"


def test_descriptor_layout_matches_header():
    # int64 m,n,p; int32 dtype,path; 3 pointers; int32 accumulate; uint32 flags
    assert ctypes.sizeof(moa.moa_gemm_desc) == 3 * 8 + 2 * 4 + 3 * 8 + 2 * 4
    assert moa.moa_gemm_desc.A.offset == 32
    assert ctypes.sizeof(moa.moa_plan_info) == 11 * 4 + 4 + 3 * 8 + 4 * 4


def test_grouped_overlap_rejected_before_launch():
    L = moa.lib()
    d1 = _desc(4, 4, 4, A=0x10000, B=0x20000, C=0x30000)
    d2 = _desc(4, 4, 4, A=0x40000, B=0x50000, C=0x30000 + 32)      # C overlaps d1's C
    arr = (moa.moa_gemm_desc * 2)(d1, d2)
    assert L.moa_gemm_grouped(arr, 2, None) == moa.MOA_ERR_INVALID
    d3 = _desc(4, 4, 4, A=0x30000, B=0x50000, C=0x60000)            # A reads d1's C
    arr = (moa.moa_gemm_desc * 2)(d1, d3)
    assert L.moa_gemm_grouped(arr, 2, None) == moa.MOA_ERR_INVALID
    bad = _desc(-1, 4, 4)
    arr = (moa.moa_gemm_desc * 2)(d1, bad)
    assert L.moa_gemm_grouped(arr, 2, None) == moa.MOA_ERR_SHAPE


def _members(shapes, flags=0):
    """Descriptors of distinct, non-overlapping (never touched) arrays."""
    out = []
    for k, (m, n, p) in enumerate(shapes):
        A = 0x100000000 + k * 3 * (1 << 26)
        out.append(_desc(m, n, p, A=A, B=A + (1 << 26), C=A + 2 * (1 << 26), flags=flags))
    return out


def test_grouped_static_rule_and_group_records(tmp_path):
    """The persistent split-BF16 kernel of a grouped launch: the static rule
    takes the block with the fewest weighted slab steps (64-row or 64-column
    blocks where 128 would be half empty), members with a column-major
    operand run singly, and an autotuner record for the members' class
    (count and median m, n, p as ceil(log2)) overrides the rule."""
    moa.moa_autotune_clear()
    q = lambda ds: moa.moa_grouped_plan_query(ds)                     # noqa: E731
    assert q(_members([(128, 300, 128)] * 8))["variant"] == 2          # 64-blocks would double the tiles
    assert q(_members([(64, 300, 256)] * 8))["variant"] == 3           # 128 rows would be half empty
    assert q(_members([(256, 300, 64)] * 8))["variant"] == 4
    c4 = [tuple(int(x) for x in s) for s in inputs.grouped_shapes(512, 32, 2048, seed=4)]
    assert q(_members(c4)) == {"variant": 2, "tuned": 0, "persistent_members": 512}
    mixed = _members([(64, 300, 256)] * 4)
    mixed[1].flags = moa.MOA_FLAG_A_COL
    assert q(mixed)["persistent_members"] == 3
    assert q(_members([(64, 300, 256)], flags=moa.MOA_FLAG_B_COL))["variant"] == -1
    f = tmp_path / "group.txt"
    f.write_text("1 16 3 6 9 8 2 0.25\n")                             # 8 members, medians 64, 300, 256
    moa.moa_autotune_load(str(f))
    assert q(_members([(64, 300, 256)] * 8)) == {"variant": 2, "tuned": 1, "persistent_members": 8}
    assert q(_members([(64, 300, 256)] * 9))["tuned"] == 0              # 9 members: another class
    g = tmp_path / "saved.txt"
    moa.moa_autotune_save(str(g))
    assert "1 16 3 6 9 8 2" in g.read_text()
    bad = tmp_path / "bad.txt"
    bad.write_text("1 16 3 6 9 8 5 0.25\n")                           # no grouped kernel 5
    with pytest.raises(moa.MoaError):
        moa.moa_autotune_load(str(bad))
    moa.moa_autotune_clear()
    assert q(_members([(64, 300, 256)] * 8))["tuned"] == 0
    L = moa.lib()
    ds = _members([(64, 300, 256)] * 2)
    arr = (moa.moa_gemm_desc * 2)(*ds)
    for v in (-2, moa.MOA_GROUPED_VARIANTS):
        assert L.moa_gemm_grouped_variant(arr, 2, v, None) == moa.MOA_ERR_INVALID
    assert L.moa_autotune_grouped(arr, 2, 0, None, None, None) == moa.MOA_ERR_INVALID


def test_serve_argument_errors_before_device():
    L = moa.lib()
    h = ctypes.c_void_p()
    assert L.moa_serve_create(None, ctypes.byref(h)) == moa.MOA_ERR_INVALID
    for cfg in (moa.moa_serve_cfg(0, 1, 1, 0, 0), moa.moa_serve_cfg(1 << 30, 0, 1, 0, 0),
                moa.moa_serve_cfg(1 << 30, 1, 0, 0, 0)):
        assert L.moa_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == moa.MOA_ERR_INVALID
    t = ctypes.c_uint64()
    assert L.moa_serve_submit(None, None, ctypes.byref(t)) == moa.MOA_ERR_INVALID
    assert L.moa_serve_poll(None, 1, None) == moa.MOA_ERR_INVALID
    assert L.moa_serve_release(None, 1) == moa.MOA_ERR_INVALID
    assert L.moa_serve_drain(None) == moa.MOA_ERR_INVALID
    assert L.moa_serve_destroy(None) == moa.MOA_OK


def test_autotune_table_save_load_and_validation(tmp_path):
    moa.moa_autotune_clear()
    f = tmp_path / "tune.txt"
    # a hand-written record: FP64 ONF, 1 term, 2^8 x 2^8 x 2^8 class -> variant 2
    f.write_text("# moa autotune v1\n0 1 1 8 8 8 2 0.5\n")
    moa.moa_autotune_load(str(f))
    q = moa.moa_plan_query(_desc(256, 256, 256, moa.MOA_F64))
    assert q["tuned"] == 1 and q["variant"] == 2
    q_other = moa.moa_plan_query(_desc(1000, 256, 256, moa.MOA_F64))   # another class
    assert q_other["tuned"] == 0
    forced = moa.moa_plan_query(_desc(256, 256, 256, moa.MOA_F64, flags=moa.MOA_FLAG_VARIANT(0)))
    assert forced["tuned"] == 0 and forced["variant"] == 0
    g = tmp_path / "out.txt"
    moa.moa_autotune_save(str(g))
    assert "0 1 1 8 8 8 2" in g.read_text()
    bad = tmp_path / "bad.txt"
    bad.write_text("0 1 1 8 8 8 9 0.5\n")                      # variant out of range
    with pytest.raises(moa.MoaError):
        moa.moa_autotune_load(str(bad))
    moa.moa_autotune_clear()
    assert moa.moa_plan_query(_desc(256, 256, 256, moa.MOA_F64))["tuned"] == 0
    assert moa.lib().moa_autotune(None, 1, None, None, None) == moa.MOA_ERR_INVALID


def _plan_variants(path, two_term):
    d = moa.moa_gemm_desc(m=64, n=64, p=64, dtype=moa.MOA_F32, path=path, A=None, B=None, C=None,
                          accumulate=0, flags=0)
    term = moa.MOA_FLAG_FP8_TWO_TERM if two_term else moa.MOA_FLAG_FP8_ONE_TERM if path == moa.MOA_PATH_FP8_SCALED else 0
    count = 0
    while True:
        d.flags = term | moa.MOA_FLAG_VARIANT(count)
        try:
            moa.moa_plan_query(d)
        except moa.MoaError:
            return count
        count += 1


RING_PATHS = [(moa.MOA_PATH_SPLIT_BF16, False), (moa.MOA_PATH_FP8_SCALED, False),
              (moa.MOA_PATH_FP8_SCALED, True), (moa.MOA_PATH_MFMA_F32, False)]


@pytest.mark.parametrize("path,two", RING_PATHS)
def test_ring_loads_stay_in_bounds_for_every_variant_and_ragged_shape(path, two):
    """Every direct load of the record ring reads inside its record array (or
    is marked dead: out of its resource's range, touching no memory), for
    blocks that overhang the operands by partial and by whole 16-row tiles."""
    shapes = [(1, 1, 1), (17, 33, 15), (130, 70, 129), (255, 16, 257), (272, 100, 48), (48, 300, 272),
              (513, 17, 769), (16, 4096, 1000), (1000, 4096, 16)]
    ran = 0
    for v in range(_plan_variants(path, two)):
        term = moa.MOA_FLAG_FP8_TWO_TERM if two else moa.MOA_FLAG_FP8_ONE_TERM if path == moa.MOA_PATH_FP8_SCALED else 0
        flags = term | moa.MOA_FLAG_VARIANT(v)
        for m, n, p in shapes:
            for extra in (0, moa.MOA_FLAG_C_COL):
                d = moa.moa_gemm_desc(m=m, n=n, p=p, dtype=moa.MOA_F32, path=path, A=None, B=None, C=None,
                                      accumulate=0, flags=flags | (extra if path != moa.MOA_PATH_MFMA_F32 else 0))
                try:
                    loads, bad = moa.moa_diag_ring_loads(d)
                except moa.MoaError as e:
                    assert e.status == moa.MOA_ERR_UNSUPPORTED      # the register-staged FP32 variant
                    continue
                assert bad == 0, (path, two, v, m, n, p, extra)
                assert loads > 0
                ran += 1
    assert ran > 0


def test_ring_load_check_refuses_non_ring_paths():
    d = moa.moa_gemm_desc(m=8, n=8, p=8, dtype=moa.MOA_F64, path=moa.MOA_PATH_ONF, A=None, B=None, C=None,
                          accumulate=0, flags=0)
    with pytest.raises(moa.MoaError) as e:
        moa.moa_diag_ring_loads(d)
    assert e.value.status == moa.MOA_ERR_UNSUPPORTED
