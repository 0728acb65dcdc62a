"""GPU parity: every path of libmoa.so against the CPU oracle, through the C ABI.

Bars (tolerances are normwise relative, ||C - R||_F / ||R||_F, FP64):
* ONF FP64 / FP32: bitwise equal to the oracle's fused multiply-add loop in
  the paper's k order (same operation sequence); FP64 also <= 1e-12 against
  the unfused oracle.
* Integer-valued inputs in {-8..8}: bitwise equal to Eq. 3 in FP64 on every
  path (all partial sums are exact integers below 2^24).
* MFMA FP32 and split-BF16: <= 1e-5 against Eq. 3 in FP64.
* Split-BF16 against the oracle's exact 3-term split product: <= 1e-6
  (FP32 accumulation only).
* FP8 against the oracle's exact product of the quantised operands: <= 1e-4.
  The FP8 matrix core sums the 64 products of one step with a hardware-defined
  accumulation that is not IEEE FP32 (measured 1.4e-5 .. 2.5e-5 on wide-range
  data; integer-valued inputs stay bit-exact); 1e-4 leaves a 4x margin. Against
  Eq. 3 the error is dominated by E4M3 rounding of the inputs and is reported
  by the benchmark.
* Conditioning (BF16 split codes, E4M3 codes, exponents): bitwise.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_11148_amd import inputs, moa

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SHAPES = [(1, 1, 1), (3, 5, 2), (31, 33, 65), (64, 64, 64), (128, 128, 128), (255, 64, 257),
          (300, 257, 520), (129, 1000, 131), (513, 96, 259)]


def variants(path, flags=0, m=300, n=300, p=300):
    """Number of block variants the planner offers for a path."""
    d = moa.moa_gemm_desc(m=m, n=n, p=p, dtype=moa.MOA_F32, path=moa.PATHS[path], A=16, B=16, C=1 << 20,
                          accumulate=0, flags=flags)
    v = 0
    while True:
        d.flags = flags | moa.MOA_FLAG_VARIANT(v)
        try:
            moa.moa_plan_query(d)
        except moa.MoaError:
            return v
        v += 1


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def run(A, B, path, dtype=None, accumulate=False, C0=None, flags=0):
    At, Bt = dev(A), dev(B)
    m, p = A.shape[0], B.shape[1]
    Ct = dev(C0) if C0 is not None else torch.full((m, p), float("nan"), dtype=At.dtype, device=DEV)
    moa.moa_gemm(At, Bt, Ct, path=path, accumulate=accumulate, flags=flags)
    torch.cuda.synchronize()
    return Ct.cpu().numpy()


@pytest.mark.parametrize("shape", SHAPES)
def test_onf_f64_bitwise_fma_order(shape):
    m, n, p = shape
    A, B = inputs.uniform_f64(m, n, p, seed=m + n + p)
    C = run(A, B, "onf")
    assert np.array_equal(C, O.gemm_f64_fma(A, B))
    assert O.rel_err(C, O.gemm_f64(A, B)) <= 1e-12


@pytest.mark.parametrize("shape", SHAPES)
def test_onf_f32_bitwise_fma_order(shape):
    m, n, p = shape
    A, B = inputs.normal_f32(m, n, p, seed=m * 7 + p)
    C = run(A, B, "onf")
    assert C.dtype == np.float32
    assert np.array_equal(C, O.gemm_f32_fma(A, B))
    assert O.rel_err(C, O.gemm_f64(A.astype(np.float64), B.astype(np.float64))) <= 1e-5


def onf_variants(dt):
    """Number of ONF block variants the planner offers for a dtype."""
    d = moa.moa_gemm_desc(m=300, n=300, p=300, dtype=moa.MOA_F64 if dt == np.float64 else moa.MOA_F32,
                          path=moa.PATHS["onf"], A=16, B=16, C=1 << 20, accumulate=0, flags=0)
    v = 0
    while True:
        d.flags = moa.MOA_FLAG_VARIANT(v)
        try:
            moa.moa_plan_query(d)
        except moa.MoaError:
            return v
        v += 1


@pytest.mark.parametrize("shape", [(200, 77, 333), (1, 16, 5), (70, 1000, 600), (130, 5, 257), (129, 8, 255),
                                   (300, 1, 140)])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_onf_every_block_size_is_bitwise_the_same(dt, shape):
    """Changing the dimension lift (block sizes) never changes a result:
    every variant (also the direct-load ring kernels: whole 8-k or 16-k
    slabs, a partial last slab, n below one slab), overwrite and accumulate,
    bitwise the
    fma-ordered oracle -- including a zero row of A over a -0 row of C,
    where one padded k step would turn -0 into +0."""
    m, n, p = shape
    A, B = inputs.uniform_f64(m, n, p, seed=5)
    A, B = A.astype(dt), B.astype(dt)
    A[0, :] = 0.0
    C0 = (np.arange(m * p).reshape(m, p) % 13 - 6).astype(dt)
    C0[0, :] = -0.0
    ref = O.gemm_f64_fma(A, B) if dt == np.float64 else O.gemm_f32_fma(A, B)
    ref_acc = O.gemm_f64_fma(A, B, C0, True) if dt == np.float64 else O.gemm_f32_fma(A, B, C0, True)
    count = onf_variants(dt)
    assert count == 5
    for v in range(count):
        fl = moa.MOA_FLAG_VARIANT(v)
        got, got_acc = run(A, B, "onf", flags=fl), run(A, B, "onf", accumulate=True, C0=C0, flags=fl)
        assert np.array_equal(got.view(np.uint64 if dt == np.float64 else np.uint32),
                              ref.view(np.uint64 if dt == np.float64 else np.uint32)), f"variant {v}"
        assert np.array_equal(got_acc.view(np.uint64 if dt == np.float64 else np.uint32),
                              ref_acc.view(np.uint64 if dt == np.float64 else np.uint32)), f"variant {v}"


@pytest.mark.parametrize("path", ["onf", "mfma_f32", "split_bf16", "fp8"])
@pytest.mark.parametrize("shape", [(5, 7, 3), (65, 129, 33), (256, 256, 256), (300, 1000, 259)])
def test_integer_valued_bit_exact_every_path(path, shape):
    m, n, p = shape
    A, B = inputs.integer_valued(m, n, p, seed=0, dtype=np.float32)
    C = run(A, B, path)
    assert np.array_equal(C.astype(np.float64), O.gemm_f64(A.astype(np.float64), B.astype(np.float64)))


def test_integer_valued_bit_exact_f64_256():
    A, B = inputs.integer_valued(256, 256, 256, seed=0, dtype=np.float64)
    assert np.array_equal(run(A, B, "onf"), O.gemm_f64(A, B))


def test_fp8_two_term_integer_exact():
    A, B = inputs.integer_valued(130, 300, 70, seed=3, dtype=np.float32)
    C = run(A, B, "fp8", flags=moa.MOA_FLAG_FP8_TWO_TERM)
    assert np.array_equal(C.astype(np.float64), O.gemm_f64(A.astype(np.float64), B.astype(np.float64)))


@pytest.mark.parametrize("shape", SHAPES)
def test_mfma_f32_tolerance(shape):
    """Every FP32 matrix-core variant within 1e-5 of Eq. 3 in FP64; the
    record-ring blocks (variants 0, 1, 3, 4) walk the same per-element
    sequence and agree bitwise; the register-staged kernel (variant 2) only
    within the bar (its k pairing inside a matrix-core step differs)."""
    m, n, p = shape
    A, B = inputs.normal_f32(m, n, p, seed=m + 3 * p)
    R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
    assert variants("mfma_f32") == 5
    out = [run(A, B, "mfma_f32", flags=moa.MOA_FLAG_VARIANT(v)) for v in range(5)]
    for C in out + [run(A, B, "mfma_f32")]:
        assert O.rel_err(C, R) <= 1e-5
    for v in (1, 3, 4):
        assert np.array_equal(out[0], out[v]), f"variant {v}"


@pytest.mark.parametrize("variant", range(4))
@pytest.mark.parametrize("shape", SHAPES)
def test_split_bf16_tolerance(shape, variant):
    if variant >= variants("split_bf16"):
        pytest.skip("no such block variant")
    m, n, p = shape
    A, B = inputs.normal_f32(m, n, p, seed=m + 5 * p)
    C = run(A, B, "split_bf16", flags=moa.MOA_FLAG_VARIANT(variant))
    R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
    assert O.rel_err(C, R) <= 1e-5
    assert O.rel_err(C, O.split_bf16_gemm(A, B)) <= 1e-6


def test_split_bf16_wide_dynamic_range():
    A, B = inputs.row_col_scaled_f32(257, 512, 300, seed=3)
    C = run(A, B, "split_bf16")
    assert O.rel_err(C, O.gemm_f64(A.astype(np.float64), B.astype(np.float64))) <= 1e-5


@pytest.mark.parametrize("shape", [(1, 1, 1), (65, 129, 33), (300, 1000, 259), (128, 256, 384)])
@pytest.mark.parametrize("two", [False, True])
def test_fp8_against_quantised_product(shape, two):
    m, n, p = shape
    A, B = inputs.row_col_scaled_f32(m, n, p, seed=m + n)
    C = run(A, B, "fp8", flags=moa.MOA_FLAG_FP8_TWO_TERM if two else moa.MOA_FLAG_FP8_ONE_TERM)
    Q = O.fp8_gemm_2term(A, B) if two else O.fp8_gemm(A, B)
    assert O.rel_err(C, Q) <= 1e-4


@pytest.mark.parametrize("two", [False, True])
def test_fp8_every_variant_same_bits(two):
    """Every block variant gives the same bits (each element sees the same
    slab sequence of matrix-core steps) and meets the quantised-product bar;
    the shape has ragged edges in m, n and p."""
    m, n, p = 300, 1000, 259
    A, B = inputs.row_col_scaled_f32(m, n, p, seed=41)
    flag = moa.MOA_FLAG_FP8_TWO_TERM if two else moa.MOA_FLAG_FP8_ONE_TERM
    outs = [run(A, B, "fp8", flags=flag | moa.MOA_FLAG_VARIANT(v)) for v in range(variants("fp8", flag))]
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    Q = O.fp8_gemm_2term(A, B) if two else O.fp8_gemm(A, B)
    assert O.rel_err(outs[0], Q) <= 1e-4


@pytest.mark.parametrize("variant", range(4))
@pytest.mark.parametrize("two", [False, True])
def test_fp8_variants_integer_exact(variant, two):
    if variant >= variants("fp8", moa.MOA_FLAG_FP8_TWO_TERM if two else moa.MOA_FLAG_FP8_ONE_TERM):
        pytest.skip("no such block variant")
    A, B = inputs.integer_valued(260, 200, 300, seed=8, dtype=np.float32)
    flag = (moa.MOA_FLAG_FP8_TWO_TERM if two else moa.MOA_FLAG_FP8_ONE_TERM) | moa.MOA_FLAG_VARIANT(variant)
    C = run(A, B, "fp8", flags=flag)
    assert np.array_equal(C.astype(np.float64), O.gemm_f64(A.astype(np.float64), B.astype(np.float64)))


def test_split_conditioning_bitwise():
    A, _ = inputs.row_col_scaled_f32(37, 1001, 1, seed=9)
    X = dev(A)
    hi = torch.empty(A.shape, dtype=torch.int16, device=DEV)
    lo = torch.empty_like(hi)
    moa.moa_split_bf16(X, hi, lo)
    torch.cuda.synchronize()
    h, l = O.bf16_split(A)
    assert np.array_equal(hi.cpu().numpy().view(np.uint16), h)
    assert np.array_equal(lo.cpu().numpy().view(np.uint16), l)


@pytest.mark.parametrize("two", [False, True])
def test_fp8_conditioning_bitwise(two):
    m, n, p = 70, 300, 90
    A, B = inputs.row_col_scaled_f32(m, n, p, seed=11)
    A[3] = 0.0                     # an all-zero row: exponent 0
    B[:, 5] = 0.0
    At, Bt = dev(A), dev(B)
    e = torch.empty(m, dtype=torch.int32, device=DEV)
    f = torch.empty(p, dtype=torch.int32, device=DEV)
    qA = torch.empty((m, n), dtype=torch.uint8, device=DEV)
    qB = torch.empty((n, p), dtype=torch.uint8, device=DEV)
    lA = torch.empty_like(qA) if two else None
    lB = torch.empty_like(qB) if two else None
    moa.moa_quantise_fp8(At, Bt, e, qA, f, qB, lA, lB, two_term=two)
    torch.cuda.synchronize()
    if two:
        rqA, rlA, re, rqB, rlB, rf = O.fp8_quantise_2term(A, B)
        assert np.array_equal(lA.cpu().numpy(), rlA)
        assert np.array_equal(lB.cpu().numpy(), rlB)
    else:
        rqA, re, rqB, rf = O.fp8_quantise(A, B)
    assert np.array_equal(e.cpu().numpy(), re)
    assert np.array_equal(f.cpu().numpy(), rf)
    assert np.array_equal(qA.cpu().numpy(), rqA)
    assert np.array_equal(qB.cpu().numpy(), rqB)


@pytest.mark.parametrize("path", ["onf", "mfma_f32", "split_bf16", "fp8"])
def test_accumulate_form(path):
    m, n, p = 70, 90, 110
    A, B = inputs.integer_valued(m, n, p, seed=2, dtype=np.float32)
    C0 = np.arange(m * p, dtype=np.float32).reshape(m, p) % 13
    C = run(A, B, path, accumulate=True, C0=C0)
    R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64), C0.astype(np.float64), accumulate=True)
    assert np.array_equal(C.astype(np.float64), R)


@pytest.mark.parametrize("path", ["onf", "mfma_f32", "split_bf16", "fp8"])
def test_empty_shared_extent(path):
    """n = 0: the empty sum assigns zero, or leaves C when accumulating."""
    m, p = 40, 50
    A = np.zeros((m, 0), np.float32)
    B = np.zeros((0, p), np.float32)
    C = run(A, B, path)
    assert np.all(C == 0)
    C0 = np.full((m, p), 3.0, np.float32)
    assert np.array_equal(run(A, B, path, accumulate=True, C0=C0), C0)


def test_empty_outputs_are_noops():
    At = torch.zeros((0, 5), device=DEV)
    Bt = torch.zeros((5, 7), device=DEV)
    Ct = torch.zeros((0, 7), device=DEV)
    moa.moa_gemm(At, Bt, Ct)


def test_error_norm_kernel():
    rng = np.random.default_rng(4)
    R = rng.standard_normal(100_003)
    X = (R + 1e-6 * rng.standard_normal(R.size)).astype(np.float32)
    out = torch.zeros(2, dtype=torch.float64, device=DEV)
    moa.moa_error_norm(dev(X), dev(R), out)
    torch.cuda.synchronize()
    num, den = out.cpu().numpy()
    ref = O.rel_err(X, R)
    assert abs(np.sqrt(num / den) - ref) <= 1e-12 * ref + 1e-300
    d = X.astype(np.float64) - R
    assert abs(num - np.sum(d * d)) <= 1e-12 * num
    assert abs(den - np.sum(R * R)) <= 1e-12 * den


def test_streams_are_respected():
    """Work issued on a side stream completes in stream order."""
    A, B = inputs.normal_f32(512, 512, 512, seed=1)
    s = torch.cuda.Stream()
    At, Bt = dev(A), dev(B)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        Ct = torch.empty((512, 512), device=DEV)
        moa.moa_gemm(At, Bt, Ct, path="onf", stream=s)
        Dt = Ct * 2
    s.synchronize()
    assert np.array_equal(Dt.cpu().numpy(), 2 * O.gemm_f32_fma(A, B))


def test_autotune_records_a_variant_and_results_stay_bitwise():
    m, n, p = 300, 257, 520
    A, B = inputs.normal_f32(m, n, p, seed=77)
    At, Bt = dev(A), dev(B)
    Ct = torch.empty((m, p), device=DEV)
    desc = moa.make_desc(At, Bt, Ct, path="onf")
    moa.moa_autotune_clear()
    try:
        plan, ms = moa.moa_autotune(desc, reps=2)
        assert plan["tuned"] == 1 and 0 <= plan["variant"] < 4 and ms > 0
        Ct.fill_(float("nan"))
        moa.moa_gemm(At, Bt, Ct, path="onf")
        torch.cuda.synchronize()
        assert np.array_equal(Ct.cpu().numpy(), O.gemm_f32_fma(A, B))
    finally:
        moa.moa_autotune_clear()


@pytest.mark.parametrize("shape", [(512, 1024, 384), (257, 4096, 129)])
def test_fp8_default_meets_the_path_bar_against_eq3(shape):
    """The scaled-FP8 path's default mode (two terms) against Eq. 3 in FP64 on
    rows of A and columns of B spanning 10^+-3: within the path's 3e-2 bar.
    The one-term mode (opt-in) is reported beside it: its error is E4M3's
    input rounding (4 significant bits), about 3.7e-2, above the bar."""
    m, n, p = shape
    A, B = inputs.row_col_scaled_f32(m, n, p, seed=m + n)
    R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
    default = run(A, B, "fp8")
    assert np.array_equal(default, run(A, B, "fp8", flags=moa.MOA_FLAG_FP8_TWO_TERM))
    err_default = O.rel_err(default, R)
    assert err_default <= 3e-2, err_default
    assert O.rel_err(default, O.fp8_gemm_2term(A, B)) <= 1e-4
    err_one = O.rel_err(run(A, B, "fp8", flags=moa.MOA_FLAG_FP8_ONE_TERM), R)
    print(f"FP8 vs Eq. 3: two terms {err_default:.3e}, one term {err_one:.3e}")
    assert 1e-2 < err_one < 6e-2
