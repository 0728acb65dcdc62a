"""Serving loop: continuous batching under an HBM budget.

* Alone vs mix: every request's result in the mixed, overlapping stream is
  bitwise the result of running the same descriptor alone through moa_gemm,
  and within the path's bar against the CPU oracle.
* Admission: at every admission instant the bytes held by admitted,
  unfinished requests stay within the budget; requests larger than the whole
  budget are refused at submit.
"""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
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


def request_bytes(r):
    m, n = r["A"].shape
    p = r["B"].shape[1]
    return 4 * (m * n + n * p + m * p) + moa.moa_plan_query(r["desc"])["workspace_bytes"]


def test_serve_budget_bounds_inflight_bytes():
    reqs = build_requests(30, seed=6, mp=(64, 512), nr=(64, 1024))
    sizes = [request_bytes(r) for r in reqs]
    budget = 3 * max(sizes)
    srv = moa.moa_serve_create(budget, slots=4, max_group=4)
    try:
        tickets = [moa.moa_serve_submit(srv, r["desc"]) for r in reqs]
        moa.moa_serve_drain(srv)
        infos = [moa.moa_serve_poll(srv, t) for t in tickets]
    finally:
        moa.moa_serve_destroy(srv)
    assert all(i["status"] == 0 for i in infos)
    # bytes are held from admission until the scheduler sees completion
    for i in infos:
        t = i["t_admit_ns"]
        held = sum(b for b, j in zip(sizes, infos) if j["t_admit_ns"] <= t < j["t_done_ns"])
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
    A = torch.zeros((256, 256), device=DEV)
    B = torch.zeros((256, 256), device=DEV)
    C = torch.zeros((256, 256), device=DEV)
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
