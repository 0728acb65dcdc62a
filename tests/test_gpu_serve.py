"""Serving loop: continuous batching under an HBM budget.

* Alone vs mix: every request's result in the mixed, overlapping stream is
  bitwise the result of running the same descriptor alone through moa_gemm,
  and within the path's bar against the CPU oracle.
* Synthetic requests: the server draws the operands on the device from the
  request's seed; the device draw is bitwise the oracle's counter-based draw,
  and each result is bitwise moa_gemm alone on the oracle's operands and
  within the path's bar against Eq. 3 in FP64 (C5-range shapes included).
* Admission: at every admission instant the bytes held by admitted,
  unfinished requests stay within the budget, and so does the server's
  device memory; requests larger than the whole budget are refused at
  submit; the batching window groups requests that arrive within it.
"""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import synthetic as SY
from paper_2306_11148_amd import inputs, moa

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def build_requests(count, seed, mp=(16, 600), nr=(16, 1200)):
    _, shapes, split = inputs.serving_stream(count, 1000.0, seed=seed, mp_range=mp, n_range=nr)
    ops = inputs.grouped_operands(shapes, seed=seed)
    reqs = []
    for (A, B), is_split in zip(ops, split):
        path = "split_bf16" if is_split else "fp8"
        flags = 0 if is_split else moa.MOA_FLAG_FP8_TWO_TERM
        At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
        Ct = torch.full((A.shape[0], B.shape[1]), float("nan"), device=DEV)
        reqs.append(dict(A=A, B=B, At=At, Bt=Bt, Ct=Ct, path=path, flags=flags,
                         desc=moa.make_desc(At, Bt, Ct, path=path, flags=flags)))
    torch.cuda.synchronize()     # operands complete before submission: the server's streams do not wait
    return reqs


def test_serve_alone_vs_mix():
    reqs = build_requests(48, seed=5)
    srv = moa.moa_serve_create(200 << 30, slots=3, max_group=8)
    try:
        tickets = []
        for k, r in enumerate(reqs):          # staggered: later requests arrive mid-flight
            tickets.append(moa.moa_serve_submit(srv, r["desc"]))
            if k % 12 == 11:
                time.sleep(0.002)
        moa.moa_serve_drain(srv)
        infos = [moa.moa_serve_poll(srv, t) for t in tickets]
    finally:
        moa.moa_serve_destroy(srv)
    assert all(i is not None and i["status"] == 0 for i in infos)
    for i in infos:
        assert i["t_submit_ns"] <= i["t_admit_ns"] <= i["t_start_ns"] <= i["t_done_ns"]
    assert max(i["group_size"] for i in infos) > 1          # requests were batched
    for r in reqs:
        alone = torch.empty_like(r["Ct"])
        moa.moa_gemm(r["At"], r["Bt"], alone, path=r["path"], flags=r["flags"])
        torch.cuda.synchronize()
        got = r["Ct"].cpu().numpy()
        assert np.array_equal(got, alone.cpu().numpy())
        if r["path"] == "split_bf16":
            R = O.gemm_f64(r["A"].astype(np.float64), r["B"].astype(np.float64))
            assert O.rel_err(got, R) <= 1e-5
        else:
            assert O.rel_err(got, O.fp8_gemm_2term(r["A"], r["B"])) <= 1e-4


def operand_bytes(r):
    m, n = r["A"].shape
    p = r["B"].shape[1]
    return 4 * (m * n + n * p + m * p)


def test_serve_budget_bounds_inflight_bytes():
    reqs = build_requests(30, seed=6, mp=(64, 512), nr=(64, 1024))
    sizes = [operand_bytes(r) + moa.moa_plan_query(r["desc"])["workspace_bytes"] for r in reqs]
    budget = 3 * max(sizes)
    srv = moa.moa_serve_create(budget, slots=4, max_group=4)
    try:
        tickets = [moa.moa_serve_submit(srv, r["desc"]) for r in reqs]
        moa.moa_serve_drain(srv)
        infos = [moa.moa_serve_poll(srv, t) for t in tickets]
        stats = moa.moa_serve_stats(srv)
    finally:
        moa.moa_serve_destroy(srv)
    assert all(i["status"] == 0 for i in infos)
    # the server's own count (operands, results, scratch) and its device memory
    assert stats["peak_held_bytes"] <= budget and stats["peak_pool_bytes"] <= budget
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    # operands are held from admission until the scheduler sees completion
    for i in infos:
        t = i["t_admit_ns"]
        held = sum(operand_bytes(r) for r, j in zip(reqs, infos) if j["t_admit_ns"] <= t < j["t_done_ns"])
        assert held <= budget
    # admission is first-come first-served
    admits = [i["t_admit_ns"] for i in infos]
    assert admits == sorted(admits)


def test_serve_release_frees_completed_tickets_only():
    reqs = build_requests(6, seed=8)
    srv = moa.moa_serve_create(200 << 30, slots=2, max_group=4)
    try:
        tickets = [moa.moa_serve_submit(srv, r["desc"]) for r in reqs]
        moa.moa_serve_drain(srv)
        for t in tickets:
            info = moa.moa_serve_poll(srv, t)
            assert info is not None and info["status"] == 0
            assert moa.moa_serve_poll(srv, t) == info          # polled again until released
            assert moa.moa_serve_release(srv, t) is True
            for call in (lambda: moa.moa_serve_poll(srv, t), lambda: moa.moa_serve_release(srv, t)):
                with pytest.raises(moa.MoaError) as ei:
                    call()
                assert ei.value.status == moa.MOA_ERR_INVALID
        # tickets are never reused after a release
        assert moa.moa_serve_submit(srv, reqs[0]["desc"]) > max(tickets)
        moa.moa_serve_drain(srv)
    finally:
        moa.moa_serve_destroy(srv)


def test_serve_refuses_request_beyond_budget_and_unknown_ticket():
    A = torch.zeros((512, 512), device=DEV)           # 3 MiB of operands and result
    B = torch.zeros((512, 512), device=DEV)
    C = torch.zeros((512, 512), device=DEV)
    srv = moa.moa_serve_create(1 << 20, slots=1, max_group=1)
    try:
        with pytest.raises(moa.MoaError) as ei:
            moa.moa_serve_submit(srv, moa.make_desc(A, B, C))
        assert ei.value.status == moa.MOA_ERR_NOMEM
        with pytest.raises(moa.MoaError) as ei:
            moa.moa_serve_poll(srv, 12345)
        assert ei.value.status == moa.MOA_ERR_INVALID
    finally:
        moa.moa_serve_destroy(srv)


# ------------------------------------------------------------ synthetic mode --

@pytest.mark.parametrize("count,offset", [(1, 0), (2, 0), (3, 1), (1023, 0), (4097, 1), (3 * 2 ** 20 + 1, 0)])
@pytest.mark.parametrize("seed", [0, 5, 2 ** 40 + 3, 2 ** 64 - 1])
def test_fill_synthetic_matches_the_oracle_draw(count, offset, seed):
    buf = torch.full((count + 2,), float("nan"), device=DEV)
    for tag in (0, 1):
        X = buf[offset:offset + count]          # offset 1: 4-byte aligned only (element stores)
        moa.moa_fill_synthetic(X, seed, tag)
        torch.cuda.synchronize()
        got = X.cpu().numpy()
        want = SY.synthetic_elements(np.arange(count), seed, tag)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
        rest = buf.cpu().numpy()
        assert np.isnan(rest[:offset]).all() and np.isnan(rest[offset + count:]).all()


def _check_synthetic(srv, t, m, n, p, path, seed, rows=None):
    info = moa.moa_serve_poll(srv, t)
    assert info is not None and info["status"] == 0
    got = np.empty((m, p), dtype=np.float32)
    moa.moa_serve_read(srv, t, got)
    A = SY.synthetic_operand(m, n, seed, 0)
    B = SY.synthetic_operand(n, p, seed, 1)
    # alone: moa_gemm on the oracle's draw of the same operands
    At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    alone = torch.empty((m, p), device=DEV)
    moa.moa_gemm(At, Bt, alone, path=path)
    torch.cuda.synchronize()
    assert np.array_equal(got, alone.cpu().numpy()), f"{m}x{n}x{p} {path}: served differs from alone"
    r = np.arange(m) if rows is None else rows
    R = O.gemm_rows_f64(A, B, r)
    bar = 1e-5 if path == "split_bf16" else 3e-2
    assert O.rel_err(got[r], R) <= bar
    if path == "fp8" and rows is None:
        assert O.rel_err(got, O.fp8_gemm_2term(A, B)) <= 1e-4
    return info


def test_serve_synthetic_alone_vs_mix_and_oracle():
    _, shapes, split = inputs.serving_stream(40, 1000.0, seed=15, mp_range=(16, 600), n_range=(16, 1200))
    reqs = [(int(m), int(n), int(p), "split_bf16" if sp else "fp8", 1000 + k)
            for k, ((m, n, p), sp) in enumerate(zip(shapes, split))]
    # C5-range products among the small ones (largest m, p and n of the workload)
    reqs[7] = (4096, 8192, 4096, "split_bf16", 77)
    reqs[23] = (4096, 2048, 1024, "fp8", 78)
    srv = moa.moa_serve_create(200 << 30, slots=3, max_group=8)
    try:
        tickets = []
        for k, (m, n, p, path, seed) in enumerate(reqs):
            tickets.append(moa.moa_serve_submit_synthetic(srv, m, n, p, path, seed))
            if k % 10 == 9:
                time.sleep(0.002)
        moa.moa_serve_drain(srv)
        infos = []
        for t, (m, n, p, path, seed) in zip(tickets, reqs):
            rows = np.random.default_rng(seed).choice(m, 48, replace=False) if m * n * p > 1e9 else None
            infos.append(_check_synthetic(srv, t, m, n, p, path, seed, rows))
        st = moa.moa_serve_stats(srv)
        assert st["held_bytes"] == sum(((m * p * 4 + 255) // 256) * 256 for m, _, p, _, _ in reqs)
        for t in tickets:
            assert moa.moa_serve_release(srv, t)
        assert moa.moa_serve_stats(srv)["held_bytes"] == 0
    finally:
        moa.moa_serve_destroy(srv)
    assert max(i["group_size"] for i in infos) > 1


def test_serve_synthetic_budget_bounds_device_memory():
    shapes = [(m, n, p) for m, n, p in inputs.serving_stream(32, 1000.0, seed=16, mp_range=(64, 512),
                                                             n_range=(64, 1024))[1].tolist()]
    one = max(4 * (m * n + n * p + m * p) for m, n, p in shapes)
    budget = 4 * one
    srv = moa.moa_serve_create(budget, slots=4, max_group=4)
    try:
        tickets = [moa.moa_serve_submit_synthetic(srv, m, n, p, "split_bf16", 500 + k)
                   for k, (m, n, p) in enumerate(shapes)]
        done = {}
        while len(done) < len(tickets):       # read and release results as they complete
            for k, t in enumerate(tickets):
                if k in done:
                    continue
                info = moa.moa_serve_poll(srv, t)
                if info is None:
                    continue
                m, n, p = shapes[k]
                if k % 8 == 0:
                    _check_synthetic(srv, t, m, n, p, "split_bf16", 500 + k)
                done[k] = info
                assert moa.moa_serve_release(srv, t)
            time.sleep(0.0005)
        st = moa.moa_serve_stats(srv)
    finally:
        moa.moa_serve_destroy(srv)
    assert all(i["status"] == 0 for i in done.values())
    assert st["peak_held_bytes"] <= budget and st["peak_pool_bytes"] <= budget
    assert st["held_bytes"] == 0 and st["completed"] == len(shapes)


def test_serve_batching_window_groups_requests():
    srv = moa.moa_serve_create(1 << 30, slots=1, max_group=6, batch_window_us=50_000)
    try:
        t0 = time.monotonic()
        tickets = [moa.moa_serve_submit_synthetic(srv, 64 + k, 96, 80, "split_bf16", 900 + k) for k in range(6)]
        assert time.monotonic() - t0 < 0.04     # all six inside the window
        moa.moa_serve_drain(srv)
        infos = [_check_synthetic(srv, t, 64 + k, 96, 80, "split_bf16", 900 + k) for k, t in enumerate(tickets)]
        assert all(i["group_size"] == 6 for i in infos)
        one = moa.moa_serve_submit_synthetic(srv, 33, 44, 55, "split_bf16", 999)
        moa.moa_serve_drain(srv)
        i = _check_synthetic(srv, one, 33, 44, 55, "split_bf16", 999)
        assert i["group_size"] == 1 and i["t_admit_ns"] - i["t_submit_ns"] >= 45_000_000
    finally:
        moa.moa_serve_destroy(srv)


def test_serve_synthetic_argument_errors():
    srv = moa.moa_serve_create(1 << 20, slots=1, max_group=1)
    try:
        for bad in (dict(m=-1, n=4, p=4, path="split_bf16"), dict(m=4, n=4, p=4, path=99)):
            with pytest.raises(moa.MoaError):
                moa.moa_serve_submit_synthetic(srv, seed=1, **bad)
        with pytest.raises(moa.MoaError) as ei:
            moa.moa_serve_submit_synthetic(srv, 4, 4, 4, "split_bf16", 1, flags=moa.MOA_FLAG_A_COL)
        assert ei.value.status == moa.MOA_ERR_INVALID
        with pytest.raises(moa.MoaError) as ei:
            moa.moa_serve_submit_synthetic(srv, 1024, 1024, 1024, "split_bf16", 1)
        assert ei.value.status == moa.MOA_ERR_NOMEM
        t = moa.moa_serve_submit_synthetic(srv, 8, 8, 8, "split_bf16", 3)
        moa.moa_serve_drain(srv)
        with pytest.raises(moa.MoaError) as ei:
            moa.moa_serve_read(srv, t, np.empty(63, dtype=np.float32))
        assert ei.value.status == moa.MOA_ERR_INVALID
        _check_synthetic(srv, t, 8, 8, 8, "split_bf16", 3)
    finally:
        moa.moa_serve_destroy(srv)
