"""Grouped products: one persistent launch for the split-BF16 members.

* Each member's result is bitwise the result of moa_gemm on the same
  descriptor (the per-element operation sequence does not depend on which
  launch or block shape produced it).
* Large groups (thousands of tiles, several claims per persistent workgroup)
  are bitwise equal to moa_gemm as well, also on a second launch that reuses
  the cached scratch.
* The batching workload at full size -- 512 products, m, n, p log-uniform in
  [32, 2048], N(0,1) FP32 -- is checked member by member against the FP64
  oracle (normwise <= 1e-5).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2306_11148_amd import inputs, moa

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def make_members(shapes, seed, path="split_bf16", accumulate=False):
    ops = inputs.grouped_operands(shapes, seed=seed)
    host, dev, descs = [], [], []
    for (A, B) in ops:
        At = torch.from_numpy(A).to(DEV)
        Bt = torch.from_numpy(B).to(DEV)
        C0 = (np.arange(A.shape[0] * B.shape[1], dtype=np.float32).reshape(A.shape[0], B.shape[1]) % 7
              if accumulate else np.full((A.shape[0], B.shape[1]), np.nan, np.float32))
        Ct = torch.from_numpy(C0).to(DEV)
        host.append((A, B, C0))
        dev.append((At, Bt, Ct))
        descs.append(moa.make_desc(At, Bt, Ct, path=path, accumulate=accumulate))
    return host, dev, descs


def singles(host, path, accumulate=False):
    out = []
    for A, B, C0 in host:
        At, Bt, Ct = (torch.from_numpy(x).to(DEV) for x in (A, B, C0))
        moa.moa_gemm(At, Bt, Ct, path=path, accumulate=accumulate)
        out.append(Ct)
    torch.cuda.synchronize()
    return [c.cpu().numpy() for c in out]


@pytest.mark.parametrize("accumulate", [False, True])
def test_grouped_split_bitwise_equals_single(accumulate):
    shapes = inputs.grouped_shapes(40, lo=1, hi=700, seed=14)
    host, dev, descs = make_members(shapes, seed=14, accumulate=accumulate)
    moa.moa_gemm_grouped(descs)
    torch.cuda.synchronize()
    ref = singles(host, "split_bf16", accumulate)
    for k, ((A, B, C0), (_, _, Ct)) in enumerate(zip(host, dev)):
        got = Ct.cpu().numpy()
        assert np.array_equal(got, ref[k]), f"member {k} shape {A.shape} x {B.shape}"
        R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64),
                       C0.astype(np.float64) if accumulate else None, accumulate)
        assert O.rel_err(got, R) <= 1e-5


@pytest.mark.parametrize("accumulate", [False, True])
@pytest.mark.parametrize("variant", range(moa.MOA_GROUPED_VARIANTS))
def test_every_grouped_kernel_bitwise_equals_single(variant, accumulate):
    """Each persistent split-BF16 kernel (block shapes 128 x 128, 64 x 128,
    128 x 64; split once or in registers) gives every member bitwise the
    single-launch result, on ragged shapes from 1 to 700."""
    shapes = inputs.grouped_shapes(40, lo=1, hi=700, seed=15)
    host, dev, descs = make_members(shapes, seed=15, accumulate=accumulate)
    moa.moa_gemm_grouped_variant(descs, variant)
    torch.cuda.synchronize()
    ref = singles(host, "split_bf16", accumulate)
    for k, ((A, B, C0), (_, _, Ct)) in enumerate(zip(host, dev)):
        got = Ct.cpu().numpy()
        assert np.array_equal(got, ref[k]), f"variant {variant} member {k} shape {A.shape} x {B.shape}"
        R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64),
                       C0.astype(np.float64) if accumulate else None, accumulate)
        assert O.rel_err(got, R) <= 1e-5


@pytest.mark.parametrize("variant", range(moa.MOA_GROUPED_VARIANTS))
def test_grouped_claims_with_few_members_and_empty_ones(variant):
    """Work-list claims by XCD segment: groups of 1, 3, 8 and 9 members (fewer
    members than segments leave segments empty; one member with m = 0 and one
    with p = 0 own no tiles) still compute every tile of every member once."""
    for count in (1, 3, 8, 9):
        shapes = [tuple(int(x) for x in s) for s in inputs.grouped_shapes(count, lo=1, hi=400, seed=40 + count)]
        if count >= 8:
            shapes[2] = (0, shapes[2][1], shapes[2][2])
            shapes[5] = (shapes[5][0], shapes[5][1], 0)
        host, dev, descs = make_members(shapes, seed=40 + count)
        moa.moa_gemm_grouped_variant(descs, variant)
        torch.cuda.synchronize()
        ref = singles(host, "split_bf16")
        for k, (_, _, Ct) in enumerate(dev):
            assert np.array_equal(Ct.cpu().numpy(), ref[k]), f"variant {variant}, {count} members, member {k}"


def test_grouped_autotune_record_drives_launches_and_groups():
    """moa_autotune_grouped times every persistent kernel on the member list
    and records the fastest for the members' class; moa_gemm_grouped and a
    prepared group then use it, and results stay bitwise the single-launch
    ones."""
    moa.moa_autotune_clear()
    shapes = inputs.grouped_shapes(24, lo=16, hi=600, seed=16)
    host, dev, descs = make_members(shapes, seed=16)
    before = moa.moa_grouped_plan_query(descs)
    assert before["tuned"] == 0 and before["persistent_members"] == len(descs)
    v, ms = moa.moa_autotune_grouped(descs, reps=2)
    assert 0 <= v < moa.MOA_GROUPED_VARIANTS and ms > 0
    after = moa.moa_grouped_plan_query(descs)
    assert after == {"variant": v, "tuned": 1, "persistent_members": len(descs)}
    ref = singles(host, "split_bf16")
    for _, _, Ct in dev:
        Ct.fill_(float("nan"))
    torch.cuda.synchronize()
    moa.moa_gemm_grouped(descs)
    torch.cuda.synchronize()
    for k, (_, _, Ct) in enumerate(dev):
        assert np.array_equal(Ct.cpu().numpy(), ref[k]), f"member {k}"
    g = moa.moa_group_create(descs)
    try:
        for _ in range(2):
            for _, _, Ct in dev:
                Ct.fill_(float("nan"))
            torch.cuda.synchronize()
            moa.moa_group_launch(g)
            torch.cuda.synchronize()
            for k, (_, _, Ct) in enumerate(dev):
                assert np.array_equal(Ct.cpu().numpy(), ref[k]), f"replay member {k}"
    finally:
        moa.moa_group_destroy(g)
        moa.moa_autotune_clear()


def test_grouped_mixed_paths_bitwise_equals_single():
    shapes = inputs.grouped_shapes(12, lo=5, hi=300, seed=21)
    paths = ["split_bf16", "onf", "fp8", "mfma_f32"] * 3
    ops = inputs.grouped_operands(shapes, seed=21)
    descs, outs, refs = [], [], []
    for (A, B), path in zip(ops, paths):
        At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
        Ct = torch.empty((A.shape[0], B.shape[1]), device=DEV)
        Rt = torch.empty_like(Ct)
        descs.append(moa.make_desc(At, Bt, Ct, path=path))
        outs.append((At, Bt, Ct))
        moa.moa_gemm(At, Bt, Rt, path=path)
        refs.append(Rt)
    moa.moa_gemm_grouped(descs)
    torch.cuda.synchronize()
    for (At, Bt, Ct), Rt in zip(outs, refs):
        assert torch.equal(Ct, Rt)


def test_grouped_empty_members_and_empty_group():
    A = torch.zeros((0, 4), device=DEV)
    B = torch.zeros((4, 3), device=DEV)
    C = torch.zeros((0, 3), device=DEV)
    moa.moa_gemm_grouped([moa.make_desc(A, B, C)])
    moa.moa_gemm_grouped([])
    A2 = torch.zeros((5, 0), device=DEV)
    B2 = torch.zeros((0, 6), device=DEV)
    C2 = torch.full((5, 6), 3.0, device=DEV)
    moa.moa_gemm_grouped([moa.make_desc(A2, B2, C2)])
    torch.cuda.synchronize()
    assert torch.all(C2 == 0)


@pytest.mark.parametrize("accumulate", [False, True])
def test_large_group_bitwise_equals_single(accumulate):
    """64 products, m, n, p log-uniform in [256, 1500] (seed 31): 2381 tiles,
    several claims per persistent workgroup."""
    shapes = inputs.grouped_shapes(64, 256, 1500, seed=31)
    host, dev, descs = make_members(shapes, seed=31, accumulate=accumulate)
    for _ in range(2):                  # a second launch reuses the cached scratch
        moa.moa_gemm_grouped(descs)
        if accumulate:
            break
    torch.cuda.synchronize()
    ref = singles(host, "split_bf16", accumulate)
    for k, ((A, B, _), (_, _, Ct)) in enumerate(zip(host, dev)):
        assert np.array_equal(Ct.cpu().numpy(), ref[k]), f"member {k} shape {A.shape} x {B.shape}"


def test_grouped_batching_workload_full_size():
    """512 products, m, n, p log-uniform in [32, 2048] (seed 4): every member
    against the FP64 oracle."""
    shapes = inputs.grouped_shapes(512, 32, 2048, seed=4)
    host, dev, descs = make_members(shapes, seed=4)
    moa.moa_gemm_grouped(descs)
    torch.cuda.synchronize()
    worst = 0.0
    for (A, B, _), (_, _, Ct) in zip(host, dev):
        R = O.gemm_f64(A.astype(np.float64), B.astype(np.float64))
        worst = max(worst, O.rel_err(Ct.cpu().numpy(), R))
    assert worst <= 1e-5, worst


def _oracle_check(A, B, got, path, fl=0):
    """A member's result against the CPU oracle at its path's bar."""
    if path == "onf":
        assert np.array_equal(got, O.gemm_f32_fma(A, B))
    elif path == "fp8":
        Q = O.fp8_gemm(A, B) if fl == moa.MOA_FLAG_FP8_ONE_TERM else O.fp8_gemm_2term(A, B)
        assert O.rel_err(got, Q) <= 1e-4
    else:
        assert O.rel_err(got, O.gemm_f64(A.astype(np.float64), B.astype(np.float64))) <= 1e-5


def test_prepared_group_graph_replays_match_single_launches():
    """Captured once, replayed three times with eager work and synchronisation
    in between; every replay is checked against single launches and every
    member against the CPU oracle."""
    shapes = inputs.grouped_shapes(18, lo=3, hi=400, seed=31)
    ops = inputs.grouped_operands(shapes, seed=31)
    paths = ["split_bf16"] * 14 + ["onf", "mfma_f32", "onf", "split_bf16"]
    members, refs = [], []
    for (A, B), path in zip(ops, paths):
        At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
        Ct = torch.empty((A.shape[0], B.shape[1]), device=DEV)
        Rt = torch.empty_like(Ct)
        moa.moa_gemm(At, Bt, Rt, path=path)
        members.append((At, Bt, Ct, moa.make_desc(At, Bt, Ct, path=path)))
        refs.append(Rt)
    torch.cuda.synchronize()
    g = moa.moa_group_create([m[3] for m in members])
    try:
        for replay in range(3):
            for _, _, Ct, _ in members:
                Ct.fill_(float("nan"))
            torch.cuda.synchronize()
            moa.moa_group_launch(g)
            torch.cuda.synchronize()
            for (_, _, Ct, _), Rt in zip(members, refs):
                assert torch.equal(Ct, Rt), f"replay {replay}"
        for (A, B), path, (_, _, Ct, _) in zip(ops, paths, members):
            _oracle_check(A, B, Ct.cpu().numpy(), path)
    finally:
        moa.moa_group_destroy(g)


def test_prepared_group_with_fp8_members_replays():
    """FP8 members of both term counts join the captured sequence; three replays
    with eager work in between all match single launches bitwise, and every
    member meets its bar against the CPU oracle."""
    shapes = inputs.grouped_shapes(16, lo=3, hi=500, seed=33)
    ops = inputs.grouped_operands(shapes, seed=33)
    flags = [moa.MOA_FLAG_FP8_ONE_TERM, moa.MOA_FLAG_FP8_TWO_TERM] * 6 + [0, 0, 0, 0]
    paths = ["fp8"] * 12 + ["split_bf16", "onf", "split_bf16", "mfma_f32"]
    members, refs = [], []
    for (A, B), path, fl in zip(ops, paths, flags):
        At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
        Ct = torch.empty((A.shape[0], B.shape[1]), device=DEV)
        Rt = torch.empty_like(Ct)
        moa.moa_gemm(At, Bt, Rt, path=path, flags=fl)
        members.append((At, Bt, Ct, moa.make_desc(At, Bt, Ct, path=path, flags=fl)))
        refs.append(Rt)
    torch.cuda.synchronize()
    g = moa.moa_group_create([m[3] for m in members])
    try:
        for replay in range(3):
            for _, _, Ct, _ in members:
                Ct.fill_(float("nan"))
            torch.cuda.synchronize()
            moa.moa_group_launch(g)
            torch.cuda.synchronize()
            for k, ((_, _, Ct, _), Rt) in enumerate(zip(members, refs)):
                assert torch.equal(Ct, Rt), f"replay {replay} member {k}"
        for (A, B), path, fl, (_, _, Ct, _) in zip(ops, paths, flags, members):
            _oracle_check(A, B, Ct.cpu().numpy(), path, fl)
    finally:
        moa.moa_group_destroy(g)


@pytest.mark.parametrize("accumulate", [False, True])
@pytest.mark.parametrize("two", [False, True])
def test_grouped_fp8_bitwise_equals_single(two, accumulate):
    """One persistent FP8 launch over ragged members (including n = 0 and
    single-row shapes): every member bitwise equal to its single launch and
    within the quantised-product bar of the oracle."""
    shapes = inputs.grouped_shapes(30, lo=1, hi=600, seed=35)
    shapes[3] = (7, 0, 9)
    shapes[4] = (1, 300, 1)
    fl = moa.MOA_FLAG_FP8_TWO_TERM if two else moa.MOA_FLAG_FP8_ONE_TERM
    rng = np.random.default_rng(36)
    host, dev, descs = [], [], []
    for (m, n, p) in shapes:
        A, B = inputs.row_col_scaled_f32(m, n, p, seed=int(rng.integers(1 << 30)))
        C0 = (np.arange(m * p, dtype=np.float32).reshape(m, p) % 5 if accumulate
              else np.full((m, p), np.nan, np.float32))
        At, Bt, Ct = (torch.from_numpy(x).to(DEV) for x in (A, B, C0))
        host.append((A, B, C0))
        dev.append(Ct)
        descs.append(moa.make_desc(At, Bt, Ct, path="fp8", accumulate=accumulate, flags=fl))
        dev.append((At, Bt))
    moa.moa_gemm_grouped(descs)
    torch.cuda.synchronize()
    outs = [dev[2 * k].cpu().numpy() for k in range(len(shapes))]
    for k, (A, B, C0) in enumerate(host):
        At, Bt = (torch.from_numpy(x).to(DEV) for x in (A, B))
        Rt = torch.from_numpy(C0).to(DEV)
        moa.moa_gemm(At, Bt, Rt, path="fp8", accumulate=accumulate, flags=fl)
        torch.cuda.synchronize()
        assert np.array_equal(outs[k], Rt.cpu().numpy()), f"member {k} shape {A.shape} x {B.shape}"
        if A.shape[1] == 0:
            assert np.array_equal(outs[k], C0 if accumulate else np.zeros_like(C0))
            continue
        Q = O.fp8_gemm_2term(A, B) if two else O.fp8_gemm(A, B)
        if accumulate:
            Q = Q + C0.astype(np.float64)
        assert O.rel_err(outs[k], Q) <= 1e-4
