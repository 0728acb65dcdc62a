#!/usr/bin/env python3
"""Benchmark of the MoA ONF matrix product on one MI355X.

Workload: C = A.B with m = n = p = 8192, FP32 row-major operands drawn
i.i.d. N(0, 1) (seeded, synthetic), resident in HBM before timing starts.

One step = one product on the split-BF16 matrix-core path: two conditioning
kernels split A's rows and B's columns into BF16 hi/lo record tiles in HBM,
then the contraction streams those records through LDS (three BF16 products
per fragment, FP32 accumulation, epilogue store): the whole path for one
input. `value` is effective TFLOP/s
= 2 N^3 / time per step. The plain ONF kernel (FP32, one fma per step in the
paper's k order) is timed on the same operands for comparison, and the FP64
oracle is timed on a bounded row sample on the host cores.

Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8192]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BF16_PEAK_TF = 2516.6       # dense BF16 matrix-core peak, MI355X
# vector FMA peaks: 256 CUs x 4 SIMDs x (32 FP32 | 16 FP64) lanes per clock x 2 flop x 2.4 GHz
FP32_VEC_PEAK_TF = 157.3
FP64_VEC_PEAK_TF = 78.6
FP8_PEAK_TF = 5033.2
COPY_CAL_BYTES = 192 * 2 ** 20   # size of the calibration copy for HBM byte counters


# path, FP8 flags, dtype and (m, n, p) of each --profile-case workload
PROFILE_CASES = {
    "split_bf16": ("split_bf16", 0, "f32", (8192, 8192, 8192)),
    "mfma_f32": ("mfma_f32", 0, "f32", (8192, 8192, 8192)),
    "onf_f32": ("onf", 0, "f32", (8192, 8192, 8192)),
    "onf_f64": ("onf", 0, "f64", (8192, 8192, 8192)),
    "onf_f64_256": ("onf", 0, "f64", (256, 256, 256)),
    "fp8_1term": ("fp8", "one", "f32", (8192, 4096, 8192)),
    "fp8_2term": ("fp8", "two", "f32", (8192, 4096, 8192)),
    # 512 products, m, n, p log-uniform [32, 2048] (seed 4): one grouped launch per step
    "grouped_c4": ("split_bf16", 0, "f32", None),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--onf-steps", type=int, default=10)
    ap.add_argument("--energy-seconds", type=float, default=2.0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=5000.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="serving: offered-load duration cap (with --serve-requests, whichever ends first)")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--ipophp", action="store_true",
                    help="time the Hadamard and Kronecker products (against the HBM roofline) and a batched "
                         "product, one JSON line per point")
    ap.add_argument("--layouts", action="store_true",
                    help="time the N x N product for every row-/column-major combination of A, B, C "
                         "(gamma_row / gamma_col), one JSON line per point")
    ap.add_argument("--split-k", type=str, default=None,
                    help="comma-separated chunk counts (0: the planner's choice, 1: unsplit): time skinny "
                         "products (few blocks of C, long k) with each, one JSON line per point")
    ap.add_argument("--serve-rates", type=str, default=None,
                    help="comma-separated offered loads (req/s): run only the serving loop at each, "
                         "one JSON line per rate")
    ap.add_argument("--serve-window", type=int, default=0,
                    help="with --serve-rates: the server's batching window in microseconds (0: none)")
    ap.add_argument("--serve-max-group", type=int, default=64,
                    help="with --serve-rates: the most requests the server puts in one grouped launch")
    ap.add_argument("--no-grouped", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--split-variants", type=str, default=None,
                    help="comma-separated N list: split-BF16 contraction and conditioning time per block "
                         "variant (square FP32 operands, seed N), two rounds, one JSON line per point")
    ap.add_argument("--block-sweep", type=str, default=None,
                    help="comma-separated N list: ONF FP64 time/energy per block size only")
    ap.add_argument("--sweep", type=str, default=None,
                    help="comma-separated N list: time/energy sweep only (one JSON line per point)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of known size (for counter scaling)")
    ap.add_argument("--profile-case", type=str, default=None, choices=sorted(PROFILE_CASES),
                    help="launch one path on its workload --warmup + --steps times and print the per-launch "
                         "times (the program rocprofv3 counter passes run)")
    ap.add_argument("--grouped-variant", type=int, default=-1,
                    help="with --profile-case grouped_c4: force this persistent kernel (-1: the planner's)")
    return ap.parse_args()


class Energy:
    """Board energy from the amd-smi accumulator (None where unavailable)."""

    def __init__(self):
        self.h = None
        self.err = None
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            hs = amdsmi.amdsmi_get_processor_handles()
            self.amdsmi = amdsmi
            self.h = hs[0] if hs else None
            if self.h is None:
                self.err = "no amd-smi processor handle"
            else:
                self.joules()
        except Exception as exc:  # amd-smi missing or not permitted
            self.h = None
            self.err = f"{type(exc).__name__}: {exc}"

    def joules(self):
        if self.h is None:
            return None
        e = self.amdsmi.amdsmi_get_energy_count(self.h)
        acc = e.get("energy_accumulator", e.get("power"))
        res = e.get("counter_resolution", 15.3)
        return float(acc) * float(res) * 1e-6

    def snapshot(self):
        out = {}
        if self.h is None:
            return out
        a = self.amdsmi
        try:
            pw = a.amdsmi_get_power_info(self.h)
            out["power_w"] = pw.get("current_socket_power", pw.get("average_socket_power"))
        except Exception:
            pass
        try:
            out["temp_hotspot_c"] = a.amdsmi_get_temp_metric(
                self.h, a.AmdSmiTemperatureType.HOTSPOT, a.AmdSmiTemperatureMetric.CURRENT)
        except Exception:
            pass
        try:
            out["gfx_clock_mhz"] = a.amdsmi_get_clock_info(self.h, a.AmdSmiClkType.GFX).get("clk")
        except Exception:
            pass
        return out


# the split-BF16 contraction kernel is built from these sources
SPLIT_KERNEL_SOURCES = ("paper_2306_11148_amd/csrc/split_bf16.hip", "paper_2306_11148_amd/csrc/ring_gemm.h",
                        "paper_2306_11148_amd/csrc/tile_common.h")


def measured_traffic(kernel_sources, record: str):
    """HBM bytes per launch from the committed counter record, or None when any
    of the kernel's source files has changed since the counters were taken
    (sha256 over the files' bytes concatenated in the listed order)."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, record)))
        h = hashlib.sha256()
        for src in kernel_sources:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != h.hexdigest() or rec.get("kernel_sources") != list(kernel_sources):
        return None
    return rec.get("hbm_bytes_per_launch")


def progress(msg: str):
    """One line on stderr as each section of the run starts."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_loop(fn, reps, torch):
    """Per-step HIP event times (ms) on the current stream, plus the total."""
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    evs[0].record()
    for r in range(reps):
        fn()
        evs[r + 1].record()
    torch.cuda.synchronize()
    per = [evs[r].elapsed_time(evs[r + 1]) for r in range(reps)]
    return per, evs[0].elapsed_time(evs[-1])


def pct(xs, q):
    s = sorted(xs)
    if not s:
        return None
    k = min(len(s) - 1, max(0, int(round(q / 100.0 * (len(s) - 1)))))
    return s[k]


def energy_per_call(fn, seconds, ms_each, energy, torch):
    """Board joules per call over about `seconds` of back-to-back calls, with
    the GFX clock and socket power sampled every 10 ms while they run."""
    if energy is None or energy.h is None:
        return None
    import threading
    reps = max(5, int(seconds * 1e3 / max(ms_each, 1e-3)))
    samples, stop = [], threading.Event()

    def sampler():
        while not stop.is_set():
            samples.append(energy.snapshot())
            time.sleep(0.01)

    torch.cuda.synchronize()
    th = threading.Thread(target=sampler)
    e0, t0 = energy.joules(), time.perf_counter()
    th.start()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    e1, t1 = energy.joules(), time.perf_counter()
    stop.set()
    th.join()

    def med(key):
        v = sorted(x[key] for x in samples if isinstance(x.get(key), (int, float)))
        return v[len(v) // 2] if v else None
    powers = [x["power_w"] for x in samples if isinstance(x.get("power_w"), (int, float))]
    out = {"joules_per_gemm": (e1 - e0) / reps, "reps": reps, "seconds": t1 - t0,
           "avg_power_w": (e1 - e0) / (t1 - t0), "median_gfx_clock_mhz": med("gfx_clock_mhz"),
           "median_power_w": med("power_w"), "median_temp_hotspot_c": med("temp_hotspot_c"),
           "clock_samples": len(samples)}
    if powers:
        # second estimate from the 10 ms power samples; the accumulator can
        # lag on some boards, moving energy between consecutive windows
        out["joules_per_gemm_sampled"] = sum(powers) / len(powers) * (t1 - t0) / reps
        if out["joules_per_gemm_sampled"] > 0 and \
                abs(out["joules_per_gemm"] / out["joules_per_gemm_sampled"] - 1.0) > 0.25:
            out["note"] = "energy accumulator and power samples disagree by more than 25%"
    return out


def cpu_baseline(A, B, C_gpu, n, target_s, onf_rows=None, precision=None):
    """The CPU leg: the FP64 oracle timed on a seeded, growing row sample of
    the same product (about target_s of oracle time), plus every error figure
    of the run (the oracle is used nowhere else in this script)."""
    import numpy as np
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    order = np.random.default_rng(1234).permutation(A.shape[0])
    rows = np.sort(order[:8])
    used = 8
    t0 = time.perf_counter()
    R = O.gemm_rows_f64(A, B, rows)
    dt = time.perf_counter() - t0
    done_rows, done_t = [rows], dt
    refs = [R]
    # grow the sample (distinct rows) until about target_s of oracle time is spent
    while done_t < target_s and used < A.shape[0]:
        want = int(min(A.shape[0] - used, max(8, len(rows) * (target_s - done_t) / max(dt, 1e-3) * 0.9)))
        more = np.sort(order[used:used + want])
        used += want
        t0 = time.perf_counter()
        refs.append(O.gemm_rows_f64(A, B, more))
        dt = time.perf_counter() - t0
        done_rows.append(more)
        done_t += dt
        rows = more
    all_rows = np.concatenate(done_rows)
    Rall = np.concatenate(refs)
    flops = 2.0 * len(all_rows) * A.shape[1] * B.shape[1]
    errs = {"split_bf16": O.rel_err(C_gpu[all_rows], Rall)}
    if onf_rows is not None:
        r_idx, got = onf_rows
        errs["onf_f32"] = O.rel_err(got, O.gemm_rows_f64(A, B, r_idx))
    if precision is not None:
        pA, pB, p_rows, kept = precision
        Rp = O.gemm_rows_f64(pA.astype(np.float64), pB.astype(np.float64), p_rows)
        errs["precision"] = {k: (O.rel_err(v, Rp), O.max_row_rel_err(v, Rp)) for k, v in kept.items()}
    return {"value": flops / done_t / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(all_rows)} seeded rows of the {n}^3 FP32 product (inputs widened to "
                      f"FP64), {done_t:.1f} s of oracle time",
            "seconds": done_t}, errs


def grouped_section(torch, moa, inputs, reps=10):
    """512 products, m, n, p log-uniform in [32, 2048] (seed 4), N(0,1) FP32
    operands drawn on the device from a seeded generator. The grouped
    autotuner first times every persistent kernel on the set and records the
    fastest (the static rule's pick is reported beside it); then one grouped
    launch, the same group prepared once and replayed as a HIP graph, and one
    launch per product are timed. The roofline of the set is the sum over
    products of max(3 x 2 m n p / BF16 peak, 4 (m n + n p + m p) bytes /
    8 TB/s)."""
    shapes = inputs.grouped_shapes(512, 32, 2048, seed=4)
    gen = torch.Generator(device="cuda").manual_seed(4)
    descs, keep = [], []
    for m, n, p in shapes:
        A = torch.randn((int(m), int(n)), generator=gen, device="cuda")
        B = torch.randn((int(n), int(p)), generator=gen, device="cuda")
        C = torch.empty((int(m), int(p)), device="cuda")
        keep.append((A, B, C))
        descs.append(moa.make_desc(A, B, C, path=moa.MOA_PATH_SPLIT_BF16))
    flops = float(sum(2.0 * m * n * p for m, n, p in shapes))
    roof_ms = float(sum(max(3 * 2.0 * m * n * p / (BF16_PEAK_TF * 1e12), 4.0 * (m * n + n * p + m * p) / 8e12)
                        for m, n, p in shapes)) * 1e3
    import ctypes
    arr = (moa.moa_gemm_desc * len(descs))(*descs)
    L, st = moa.lib(), torch.cuda.current_stream().cuda_stream
    moa.moa_autotune_clear()
    static_variant = moa.moa_grouped_plan_query(descs)["variant"]
    variant_ms = {}
    for v in range(moa.MOA_GROUPED_VARIANTS):
        def run_v(v=v):
            if L.moa_gemm_grouped_variant(arr, len(descs), v, st) != 0:
                raise RuntimeError(moa.moa_last_error())
        run_v()
        variant_ms[v] = round(timed_loop(run_v, reps, torch)[1] / reps, 4)
    tuned_variant, tuned_ms = moa.moa_autotune_grouped(descs, reps=reps)
    plan = moa.moa_grouped_plan_query(descs)
    group = moa.moa_group_create(descs)          # built with the tuned kernel

    def grouped():
        if L.moa_gemm_grouped(arr, len(descs), st) != 0:
            raise RuntimeError(moa.moa_last_error())

    def replay():
        if L.moa_group_launch(ctypes.c_void_p(group), st) != 0:
            raise RuntimeError(moa.moa_last_error())

    def singles():
        for d in descs:
            if L.moa_gemm(ctypes.byref(d), st) != 0:
                raise RuntimeError(moa.moa_last_error())
    try:
        for _ in range(2):
            grouped()
            replay()
            singles()
        per_g, tot_g = timed_loop(grouped, reps, torch)
        per_r, tot_r = timed_loop(replay, reps, torch)
        per_s, tot_s = timed_loop(singles, reps, torch)
        moa.moa_trace_read(reset=True)
        moa.moa_trace_enable(True)
        timed_loop(grouped, reps, torch)
        moa.moa_trace_enable(False)
        traced = moa.moa_trace_read(reset=True)
    finally:
        moa.moa_group_destroy(group)
        moa.moa_autotune_clear()
    ms_g, ms_r, ms_s = tot_g / reps, tot_r / reps, tot_s / reps
    n_k, t_k = traced.get("split_grouped", (0, 0.0))
    del keep
    best = min(ms_g, ms_r)
    return {"workload": "512 products, m,n,p log-uniform [32,2048], split-BF16, seed 4",
            "flop": flops, "grouped_ms": round(ms_g, 4), "graph_replay_ms": round(ms_r, 4),
            "per_gemm_launches_ms": round(ms_s, 4),
            "grouped_tflops": round(flops / ms_g / 1e9, 2), "graph_replay_tflops": round(flops / ms_r / 1e9, 2),
            "per_gemm_tflops": round(flops / ms_s / 1e9, 2),
            "speedup": round(ms_s / best, 3),
            "persistent_kernel": {"static_rule": static_variant, "autotuned": tuned_variant,
                                  "used": plan["variant"], "tuned": plan["tuned"],
                                  "autotune_best_ms": round(tuned_ms, 4),
                                  "ms_by_kernel": variant_ms,
                                  "kernels": {0: "128x128 split once, 3/CU", 1: "128x128 split once, 2 plane sets, 2/CU",
                                              2: "128x128 split in registers, 2/CU", 3: "64x128 split once, 4/CU",
                                              4: "128x64 split once, 4/CU"}},
            "contraction_kernel_ms": round(t_k / n_k, 4) if n_k else None,
            "roofline": {"bound": "sum over products of max(matrix-core, HBM) time", "ideal_ms": round(roof_ms, 4),
                         "frac": round(roof_ms / best, 4)}}


def serving_section(torch, moa, inputs, rate, seconds, max_requests, seed=5, verify_share=0.01, window_us=0,
                    max_group=64):
    """Open-loop Poisson arrivals at `rate` req/s: min(rate * seconds,
    max_requests) synthetic requests, m, p log-uniform [64, 4096], n
    log-uniform [64, 8192], 70% split-BF16 / 30% two-term FP8. Each request is
    (shape, path, seed): the server takes its operands and result from its
    budgeted pool and draws A and B on the device at admission. Latency =
    completion - scheduled arrival (requests are submitted at their scheduled
    times, late or not, so no coordinated omission); the first 5% are
    discarded. The client releases each result as it completes, except a
    seeded share of the requests whose C stays in the pool until the timed
    loop has ended; then a 16 x 16 sub-block of each (sampled rows and
    columns) is read for the CPU leg to check against the oracle."""
    import numpy as np
    count = max(1, min(int(rate * seconds), max_requests))
    t_arr, shapes, split = inputs.serving_stream(count, rate, seed=seed)
    rng = np.random.default_rng(seed + 99)
    verify = set(rng.choice(count, size=max(1, int(np.ceil(verify_share * count))), replace=False).tolist())
    seed_of = lambda q: (seed << 32) + q      # noqa: E731
    path_of = lambda q: "split_bf16" if split[q] else "fp8"   # noqa: E731
    budget = 200 << 30
    reserve = 16 << 30       # taken at creation: no allocation while requests run
    srv = moa.moa_serve_create(budget, slots=4, max_group=max_group, batch_window_us=window_us,
                               pool_reserve_bytes=reserve)
    kept, infos, sched_ns = {}, [None] * count, [0] * count
    try:
        # untimed warm-up: the first shapes once through the server (code
        # objects, pool chunks, staging buffers)
        warm = [moa.moa_serve_submit_synthetic(srv, *(int(x) for x in shapes[q]), path_of(q), 1 << 62 | q)
                for q in range(min(count, 64))]
        moa.moa_serve_drain(srv)
        for t in warm:
            moa.moa_serve_release(srv, t)
        pending = []                         # (ticket, q) in submission order
        held = []                            # finished requests kept for the CPU check

        def reap(block=False):
            while pending:
                t, q = pending[0]
                info = moa.moa_serve_poll(srv, t)
                if info is None:
                    if not block:
                        return
                    continue
                if q in verify:
                    held.append((t, q))      # read after the timed loop; its C stays in the pool until then
                else:
                    moa.moa_serve_release(srv, t)
                infos[q] = info
                pending.pop(0)
        flops = 0.0
        t0 = time.monotonic_ns() + 20_000_000
        for q in range(count):
            m, n, p = (int(x) for x in shapes[q])
            due = t0 + int(t_arr[q] * 1e9)
            while time.monotonic_ns() < due:
                reap()
            pending.append((moa.moa_serve_submit_synthetic(srv, m, n, p, path_of(q), seed_of(q),
                                                           flags=0 if split[q] else moa.MOA_FLAG_FP8_TWO_TERM), q))
            sched_ns[q] = due
            flops += 2.0 * m * n * p
        moa.moa_serve_drain(srv)
        reap(block=True)
        stats = moa.moa_serve_stats(srv)
        for t, q in held:
            m, n, p = (int(x) for x in shapes[q])
            C = np.empty((m, p), dtype=np.float32)
            moa.moa_serve_read(srv, t, C)
            moa.moa_serve_release(srv, t)
            r = np.random.default_rng(q)
            rows = np.sort(r.choice(m, min(m, 16), replace=False))
            cols = np.sort(r.choice(p, min(p, 16), replace=False))
            kept[q] = (m, n, p, path_of(q), seed_of(q), rows, cols, C[np.ix_(rows, cols)].copy())
    finally:
        moa.moa_serve_destroy(srv)
    lat = np.array([(i["t_done_ns"] - s) / 1e6 for i, s in zip(infos, sched_ns)])
    skip = int(0.05 * count)
    body = lat[skip:]
    span = (max(i["t_done_ns"] for i in infos) - sched_ns[0]) / 1e9
    bad = sum(1 for i in infos if i["status"] != 0)
    groups = np.array([i["group_size"] for i in infos])
    out = {"rate_req_per_s": rate, "batch_window_us": window_us, "max_group": max_group, "requests": count,
           "seconds": round(span, 3),
           "latency_ms": {"p50": round(float(np.percentile(body, 50)), 3),
                          "p99": round(float(np.percentile(body, 99)), 3),
                          "mean": round(float(body.mean()), 3)},
           "tflops": round(flops / span / 1e12, 2), "failed": bad,
           "mean_group_size": round(float(groups.mean()), 2),
           "mix": "70% split-BF16 / 30% two-term FP8, synthetic requests (operands drawn on the device "
                  "at admission), HBM budget 200 GB, 4 slots, groups <= " + str(max_group),
           "first_5pct_discarded": skip,
           "device_memory": {"budget_bytes": budget, "pool_reserve_bytes": reserve,
                             "peak_pool_bytes": stats["peak_pool_bytes"],
                             "peak_held_bytes": stats["peak_held_bytes"]},
           "verified": None}
    return out, kept


def cpu_verify_serving(kept):
    """The CPU leg's check of the served results: for each kept request, the
    oracle's draw of the sampled rows of A and columns of B and Eq. 3 in FP64
    on that sub-block; normwise error per request against the path's bar."""
    import numpy as np
    from oracle import oracle as O
    from oracle import synthetic as SY
    errs = {"split_bf16": [], "fp8": []}
    for m, n, p, path, sd, rows, cols, got in kept.values():
        A = SY.synthetic_operand(m, n, sd, 0, row_index=rows)
        idx = np.arange(n, dtype=np.int64)[:, None] * p + np.asarray(cols, dtype=np.int64)[None, :]
        B = SY.synthetic_elements(idx, sd, 1).reshape(n, len(cols))
        errs[path].append(O.rel_err(got, O.gemm_f64(A.astype(np.float64), B.astype(np.float64))))
    bars = {"split_bf16": 1e-5, "fp8": 3e-2}
    out = {"requests": len(kept), "block": "16 x 16 sampled rows x columns of C per request"}
    for k, v in errs.items():
        if v:
            out[k] = {"count": len(v), "max_err": float(max(v)), "median_err": float(np.median(v)),
                      "bar": bars[k], "all_within_bar": bool(max(v) <= bars[k])}
    return out


def fp64_sections(torch, moa, inputs, N, steps, energy):
    """The paper's own precision on the plain ONF kernel: the N x N x N FP64
    product (A, B uniform[-1, 1), seed N) with its joules per product, and
    the 256^3 FP64 product (seed 0) plus its integer-valued copy (entries in
    {-8..8}). Results are kept for the CPU leg's error figures."""
    import ctypes
    import numpy as np
    L, st = moa.lib(), torch.cuda.current_stream().cuda_stream
    out, keep = {}, {}

    def timed(d, reps):
        def f():
            if L.moa_gemm(ctypes.byref(d), st) != 0:
                raise RuntimeError(moa.moa_last_error())
        f()
        per, tot = timed_loop(f, reps, torch)
        return f, per, tot / reps

    A_h, B_h = inputs.uniform_f64(N, N, N, seed=N)
    A, B = torch.from_numpy(A_h).cuda(), torch.from_numpy(B_h).cuda()
    C = torch.empty((N, N), dtype=torch.float64, device="cuda")
    d = moa.make_desc(A, B, C, path=moa.MOA_PATH_ONF)
    f, per, ms = timed(d, steps)
    tf = 2.0 * N ** 3 / ms / 1e9
    rows = np.arange(0, N, max(1, N // 32))
    keep["onf_f64"] = (A_h, B_h, rows, C.cpu().numpy()[rows])
    out["onf_f64"] = {"workload": f"{N}^3 FP64, A, B uniform[-1,1), seed {N}", "ms": round(ms, 3),
                      "tflops": round(tf, 2), "roofline": {"bound": "alu", "achieved": round(tf, 2),
                                                           "peak": FP64_VEC_PEAK_TF, "unit": "TFLOP/s",
                                                           "frac": round(tf / FP64_VEC_PEAK_TF, 4)},
                      "p50_ms": round(pct(per, 50), 3), "p99_ms": round(pct(per, 99), 3),
                      "plan": moa.moa_plan_query(d), "normwise_err_sampled": None,
                      "energy": energy_per_call(f, 2.0, ms, energy, torch) if energy else None}
    del A, B, C
    A_h, B_h = inputs.uniform_f64(256, 256, 256, seed=0)
    Ai_h, Bi_h = inputs.integer_valued(256, 256, 256, seed=0)
    A, B, Ai, Bi = (torch.from_numpy(x).cuda() for x in (A_h, B_h, Ai_h, Bi_h))
    C, Ci = (torch.empty((256, 256), dtype=torch.float64, device="cuda") for _ in range(2))
    d, di = moa.make_desc(A, B, C, path=moa.MOA_PATH_ONF), moa.make_desc(Ai, Bi, Ci, path=moa.MOA_PATH_ONF)
    _, per, ms = timed(d, 200)
    timed(di, 1)
    torch.cuda.synchronize()
    keep["c1"] = (A_h, B_h, C.cpu().numpy(), Ai_h, Bi_h, Ci.cpu().numpy())
    out["c1_256_f64"] = {"workload": "256^3 FP64, A, B uniform[-1,1), seed 0; integer-valued copy {-8..8}",
                         "ms": round(ms, 4), "tflops": round(2.0 * 256 ** 3 / ms / 1e9, 3),
                         "p50_ms": round(pct(per, 50), 4), "p99_ms": round(pct(per, 99), 4),
                         "bound": "launch latency (3.4e7 flop: 0.43 us at the FP64 peak)",
                         "normwise_err": None, "integer_bitwise": None}
    return out, keep


def cpu_check_fp64(keep):
    """CPU leg: errors of the FP64 products against the FP64 oracle."""
    import numpy as np
    from oracle import oracle as O
    A_h, B_h, rows, got = keep["onf_f64"]
    A2, B2, C2, Ai, Bi, Ci = keep["c1"]
    return {"onf_f64_sampled": O.rel_err(got, O.gemm_rows_f64(A_h, B_h, rows)),
            "c1": O.rel_err(C2, O.gemm_f64(A2, B2)),
            "c1_integer_bitwise": bool(np.array_equal(Ci, O.gemm_f64(Ai, Bi)))}


def precision_section(torch, moa, inputs, reps=5):
    """m=8192, n=4096, p=8192, FP32 inputs N(0,1)*10^U(-3,3) per row of A and
    column of B (seed 3): every path timed; 48 seeded rows of each result are
    kept for the CPU leg, which measures their error against the oracle."""
    import ctypes
    import numpy as np
    m, n, p = 8192, 4096, 8192
    A_h, B_h = inputs.row_col_scaled_f32(m, n, p, seed=3)
    A = torch.from_numpy(A_h).cuda()
    B = torch.from_numpy(B_h).cuda()
    C = torch.empty((m, p), device="cuda")
    rows = np.sort(np.random.default_rng(33).choice(m, 48, replace=False))
    out = {"workload": "m=8192 n=4096 p=8192, N(0,1)*10^U(-3,3) per row of A / column of B, seed 3",
           "error": "normwise and worst row-wise relative error vs the FP64 oracle on 48 seeded "
                    "rows (computed in the CPU leg)"}
    kept = {}
    paths = [("onf_f32", moa.MOA_PATH_ONF, 0), ("mfma_f32", moa.MOA_PATH_MFMA_F32, 0),
             ("split_bf16", moa.MOA_PATH_SPLIT_BF16, 0), ("fp8_1term", moa.MOA_PATH_FP8_SCALED, moa.MOA_FLAG_FP8_ONE_TERM),
             ("fp8_2term", moa.MOA_PATH_FP8_SCALED, moa.MOA_FLAG_FP8_TWO_TERM)]
    L, st = moa.lib(), torch.cuda.current_stream().cuda_stream
    for name, path, flags in paths:
        d = moa.make_desc(A, B, C, path=path, flags=flags)

        def f():
            if L.moa_gemm(ctypes.byref(d), st) != 0:
                raise RuntimeError(moa.moa_last_error())
        f()
        torch.cuda.synchronize()
        kept[name] = C.cpu().numpy()[rows]
        _, tot = timed_loop(f, reps, torch)
        ms = tot / reps
        out[name] = {"ms": round(ms, 4), "tflops": round(2.0 * m * n * p / ms / 1e9, 2),
                     "normwise_err": None, "max_row_rel_err": None}
    return out, (A_h, B_h, rows, kept)


def sweep(args, torch, moa, inputs):
    """Time and joules per product against N for the square FP32 workload, per
    path (the paper's time/energy-versus-N axes), one JSON line per point."""
    energy = Energy()
    for N in [int(x) for x in args.sweep.split(",")]:
        gen = torch.Generator(device="cuda").manual_seed(N)
        A = torch.randn((N, N), generator=gen, device="cuda")
        B = torch.randn((N, N), generator=gen, device="cuda")
        C = torch.empty((N, N), device="cuda")
        for name, path, flags in (("onf_f32", moa.MOA_PATH_ONF, 0),
                                  ("mfma_f32", moa.MOA_PATH_MFMA_F32, 0),
                                  ("split_bf16", moa.MOA_PATH_SPLIT_BF16, 0),
                                  ("fp8_1term", moa.MOA_PATH_FP8_SCALED, moa.MOA_FLAG_FP8_ONE_TERM),
                                  ("fp8_2term", moa.MOA_PATH_FP8_SCALED, moa.MOA_FLAG_FP8_TWO_TERM)):
            d = moa.make_desc(A, B, C, path=path, flags=flags)
            L, st = moa.lib(), torch.cuda.current_stream().cuda_stream
            import ctypes

            def f():
                if L.moa_gemm(ctypes.byref(d), st) != 0:
                    raise RuntimeError(moa.moa_last_error())
            f()
            reps = max(3, min(200, int(200.0 / (2.0 * N ** 3 / 1e11))))
            per, tot = timed_loop(f, reps, torch)
            ms = tot / reps
            e = energy_per_call(f, args.energy_seconds, ms, energy, torch)
            print(json.dumps({"sweep": "square FP32", "N": N, "path": name, "ms": round(ms, 4),
                              "tflops": round(2.0 * N ** 3 / ms / 1e9, 2),
                              "p50_ms": round(pct(per, 50), 4), "p99_ms": round(pct(per, 99), 4),
                              "energy": e}), flush=True)
        del A, B, C


def ipophp_section(torch, moa):
    """Hadamard (m x n), Kronecker (A m x n, B p x q) and batched products.
    The first two are HBM-bound: achieved = algorithmic bytes (read A and B,
    write C; C also read when accumulating) / time, against 8 TB/s."""
    gen = torch.Generator(device="cuda").manual_seed(21)
    for dt, es in ((torch.float32, 4), (torch.float64, 8)):
        N = 8192
        A = torch.randn((N, N), generator=gen, device="cuda", dtype=dt)
        B = torch.randn((N, N), generator=gen, device="cuda", dtype=dt)
        C = torch.empty((N, N), device="cuda", dtype=dt)
        for acc in (False, True):
            moa.moa_hadamard(A, B, C, accumulate=acc)
            per, tot = timed_loop(lambda: moa.moa_hadamard(A, B, C, accumulate=acc), 20, torch)
            ms = tot / 20
            nbytes = (4 if acc else 3) * N * N * es
            print(json.dumps({"ipophp": {"op": "hadamard", "dtype": str(dt).split(".")[-1], "m": N, "n": N,
                                         "accumulate": acc, "ms": round(ms, 4), "bytes": nbytes,
                                         "GBps": round(nbytes / ms / 1e6, 1),
                                         "frac_of_8TBps": round(nbytes / ms / 1e6 / 8000.0, 3)}}), flush=True)
        del A, B, C
        a = torch.randn((64, 64), generator=gen, device="cuda", dtype=dt)
        b = torch.randn((128, 128), generator=gen, device="cuda", dtype=dt)
        K = torch.empty((8192, 8192), device="cuda", dtype=dt)
        moa.moa_kronecker(a, b, K)
        per, tot = timed_loop(lambda: moa.moa_kronecker(a, b, K), 20, torch)
        ms = tot / 20
        nbytes = 8192 * 8192 * es + (64 * 64 + 128 * 128) * es
        print(json.dumps({"ipophp": {"op": "kronecker", "dtype": str(dt).split(".")[-1], "A": [64, 64],
                                     "B": [128, 128], "ms": round(ms, 4), "bytes": nbytes,
                                     "GBps": round(nbytes / ms / 1e6, 1),
                                     "frac_of_8TBps": round(nbytes / ms / 1e6 / 8000.0, 3)}}), flush=True)
        del K
    batch, m, n, p = 64, 512, 512, 512
    A = torch.randn((batch, m, n), generator=gen, device="cuda")
    B = torch.randn((batch, n, p), generator=gen, device="cuda")
    C = torch.empty((batch, m, p), device="cuda")
    moa.moa_gemm_batched(A, B, C, path="split_bf16")
    per, tot = timed_loop(lambda: moa.moa_gemm_batched(A, B, C, path="split_bf16"), 20, torch)
    ms = tot / 20
    print(json.dumps({"ipophp": {"op": "batched", "path": "split_bf16", "batch": batch, "m": m, "n": n, "p": p,
                                 "ms": round(ms, 4), "tflops": round(2.0 * batch * m * n * p / ms / 1e9, 2)}}),
          flush=True)


def layout_sweep(args, torch, moa):
    """Time per N x N product for each layout of A, B and C (row-major or
    column-major, the latter passed as the transpose of a contiguous tensor)."""
    import ctypes
    import itertools
    N = args.n
    L, st = moa.lib(), torch.cuda.current_stream().cuda_stream
    gen = torch.Generator(device="cuda").manual_seed(N)
    A0 = torch.randn((N, N), generator=gen, device="cuda")
    B0 = torch.randn((N, N), generator=gen, device="cuda")
    C0 = torch.empty((N, N), device="cuda")
    for name, path, flags in (("split_bf16", moa.MOA_PATH_SPLIT_BF16, 0),
                              ("fp8_1term", moa.MOA_PATH_FP8_SCALED, moa.MOA_FLAG_FP8_ONE_TERM),
                              ("mfma_f32", moa.MOA_PATH_MFMA_F32, 0),
                              ("onf_f32", moa.MOA_PATH_ONF, 0)):
        for ac, bc, cc in itertools.product([False, True], repeat=3):
            d = moa.make_desc(A0.t() if ac else A0, B0.t() if bc else B0, C0.t() if cc else C0,
                              path=path, flags=flags)

            def f():
                if L.moa_gemm(ctypes.byref(d), st) != 0:
                    raise RuntimeError(moa.moa_last_error())
            f()
            reps = 3 if name == "onf_f32" else 20
            per, tot = timed_loop(f, reps, torch)
            ms = tot / reps
            print(json.dumps({"layout_sweep": {"N": N, "path": name, "A": "col" if ac else "row",
                                               "B": "col" if bc else "row", "C": "col" if cc else "row",
                                               "ms": round(ms, 4), "tflops": round(2.0 * N ** 3 / ms / 1e9, 2)}}),
                  flush=True)


def split_k_sweep(args, torch, moa, inputs):
    """Skinny products whose m x p blocks cannot fill the 256 CUs: time per
    product with the k walk split into c chunks (c = 1: no split)."""
    import ctypes
    L, st = moa.lib(), torch.cuda.current_stream().cuda_stream
    for (m, n, p) in ((256, 65536, 256), (512, 32768, 512), (1024, 16384, 1024)):
        gen = torch.Generator(device="cuda").manual_seed(m + n + p)
        A = torch.randn((m, n), generator=gen, device="cuda")
        B = torch.randn((n, p), generator=gen, device="cuda")
        C = torch.empty((m, p), device="cuda")
        for name, path, base in (("split_bf16", moa.MOA_PATH_SPLIT_BF16, 0),
                                 ("fp8_2term", moa.MOA_PATH_FP8_SCALED, moa.MOA_FLAG_FP8_TWO_TERM)):
            for c in [int(x) for x in args.split_k.split(",")]:
                # c = 0: the planner's choice; c = 1: kept whole; c > 1: c chunks asked for
                d = moa.make_desc(A, B, C, path=path, flags=base | (moa.MOA_FLAG_SPLIT_K(c) if c >= 1 else 0))
                plan = moa.moa_plan_query(d)

                def f():
                    if L.moa_gemm(ctypes.byref(d), st) != 0:
                        raise RuntimeError(moa.moa_last_error())
                for _ in range(3):
                    f()
                per, tot = timed_loop(f, 20, torch)
                ms = tot / 20
                print(json.dumps({"split_k_sweep": {"m": m, "n": n, "p": p, "path": name, "asked": c or "planner",
                                                    "chunks": plan["split_k"],
                                                    "workgroups": plan["workgroups"], "ms": round(ms, 4),
                                                    "tflops": round(2.0 * m * n * p / ms / 1e9, 2),
                                                    "p50_ms": round(pct(per, 50), 4)}}), flush=True)
        del A, B, C


def block_sweep(args, torch, moa):
    """The paper's experiment on this GPU: time and joules per product against
    N for every block size of the plain ONF kernel in FP64 (one JSON line per
    point). Block sizes are the planner's ONF instantiations, the first being
    the static rule's 32 x 32 doubles."""
    import ctypes
    energy = Energy()
    L, st = moa.lib(), torch.cuda.current_stream().cuda_stream
    for N in [int(x) for x in args.block_sweep.split(",")]:
        gen = torch.Generator(device="cuda").manual_seed(N)
        A = torch.rand((N, N), generator=gen, device="cuda", dtype=torch.float64) * 2 - 1
        B = torch.rand((N, N), generator=gen, device="cuda", dtype=torch.float64) * 2 - 1
        C = torch.empty((N, N), device="cuda", dtype=torch.float64)
        for v in range(5):
            d = moa.make_desc(A, B, C, path=moa.MOA_PATH_ONF, flags=moa.MOA_FLAG_VARIANT(v))
            plan = moa.moa_plan_query(d)

            def f():
                if L.moa_gemm(ctypes.byref(d), st) != 0:
                    raise RuntimeError(moa.moa_last_error())
            f()
            reps = max(2, min(100, int(0.5 / (2.0 * N ** 3 / 5e13))))
            per, tot = timed_loop(f, reps, torch)
            ms = tot / reps
            e = energy_per_call(f, min(args.energy_seconds, 1.0), ms, energy, torch)
            print(json.dumps({"block_sweep": "ONF FP64", "N": N, "variant": v,
                              "staging": "direct-to-LDS ring" if plan["tile_k"] == 8 else "registers",
                              "block": [plan["tile_m"], plan["tile_n"]],
                              "components": plan["tile_m"] * plan["tile_n"], "ms": round(ms, 4),
                              "tflops": round(2.0 * N ** 3 / ms / 1e9, 3), "energy": e}), flush=True)
        del A, B, C


def split_variants(args, torch, moa):
    """Kernel times of every split-BF16 block variant against N (library trace:
    HIP events on the launch stream), two rounds over the list, so that the
    spread between rounds shows alongside the differences between variants."""
    d0 = moa.moa_gemm_desc(m=1024, n=1024, p=1024, dtype=moa.MOA_F32, path=moa.MOA_PATH_SPLIT_BF16,
                           A=16, B=16, C=1 << 24, accumulate=0, flags=0)
    count = 0
    while True:
        d0.flags = moa.MOA_FLAG_VARIANT(count)
        try:
            moa.moa_plan_query(d0)
        except moa.MoaError:
            break
        count += 1
    for rnd in range(2):
        for N in [int(x) for x in args.split_variants.split(",")]:
            gen = torch.Generator(device="cuda").manual_seed(N)
            A = torch.randn((N, N), generator=gen, device="cuda")
            B = torch.randn((N, N), generator=gen, device="cuda")
            C = torch.empty((N, N), device="cuda")
            default = moa.moa_plan_query(moa.make_desc(A, B, C, path=moa.MOA_PATH_SPLIT_BF16))["variant"]
            for v in range(count):
                fl = moa.MOA_FLAG_VARIANT(v)
                plan = moa.moa_plan_query(moa.make_desc(A, B, C, path=moa.MOA_PATH_SPLIT_BF16, flags=fl))
                for _ in range(3):
                    moa.moa_gemm(A, B, C, path="split_bf16", flags=fl)
                torch.cuda.synchronize()
                moa.moa_trace_enable(True)
                moa.moa_trace_read(reset=True)
                reps = max(5, min(50, int(2e12 / N ** 3)))
                for _ in range(reps):
                    moa.moa_gemm(A, B, C, path="split_bf16", flags=fl)
                torch.cuda.synchronize()
                st = moa.moa_trace_read(reset=True)
                moa.moa_trace_enable(False)
                k_ms = st["split_bf16"][1] / st["split_bf16"][0]
                p_ms = st["split_pack"][1] / st["split_pack"][0]
                print(json.dumps({"split_variants": rnd, "N": N, "variant": v, "default": v == default,
                                  "block": [plan["tile_m"], plan["tile_n"]], "wave": [plan["wave_m"], plan["wave_n"]],
                                  "kernel_ms": round(k_ms, 4), "pack_ms": round(p_ms, 4),
                                  "kernel_tflops_issued": round(3 * 2.0 * N ** 3 / k_ms / 1e9, 1)}), flush=True)
            del A, B, C


def profile_grouped(args, torch, moa):
    """--profile-case grouped_c4: the batching workload's grouped launch
    (the planner's persistent kernel, or --grouped-variant's), --warmup
    untimed and --steps timed."""
    import ctypes
    from paper_2306_11148_amd import inputs
    shapes = inputs.grouped_shapes(512, 32, 2048, seed=4)
    gen = torch.Generator(device="cuda").manual_seed(4)
    descs, keep = [], []
    for m, n, p in shapes:
        A = torch.randn((int(m), int(n)), generator=gen, device="cuda")
        B = torch.randn((int(n), int(p)), generator=gen, device="cuda")
        C = torch.empty((int(m), int(p)), device="cuda")
        keep.append((A, B, C))
        descs.append(moa.make_desc(A, B, C, path=moa.MOA_PATH_SPLIT_BF16))
    arr = (moa.moa_gemm_desc * len(descs))(*descs)
    L, st = moa.lib(), torch.cuda.current_stream().cuda_stream

    def f():
        if L.moa_gemm_grouped_variant(arr, len(descs), args.grouped_variant, st) != 0:
            raise RuntimeError(moa.moa_last_error())
    for _ in range(args.warmup):
        f()
    per, tot = timed_loop(f, args.steps, torch)
    flop = float(sum(2.0 * m * n * p for m, n, p in shapes))
    print(json.dumps({"profile_case": "grouped_c4", "members": len(descs), "flop": flop,
                      "plan": moa.moa_grouped_plan_query(descs), "forced_variant": args.grouped_variant,
                      "launches": args.steps,
                      "ms_per_launch": round(tot / args.steps, 4), "per_launch_ms": [round(x, 4) for x in per],
                      "tflops": round(flop / (tot / args.steps) / 1e9, 2)}), flush=True)
    del keep


def profile_case(args, torch, moa):
    """One path on its workload, --warmup untimed and --steps timed launches
    (HIP events on the launch stream), for counter and trace passes; the
    copy-calibration copy runs last when asked for."""
    import ctypes
    name = args.profile_case
    if name == "grouped_c4":
        return profile_grouped(args, torch, moa)
    path, fp8, dt, (m, n, p) = PROFILE_CASES[name]
    dtype = torch.float64 if dt == "f64" else torch.float32
    gen = torch.Generator(device="cuda").manual_seed(n)
    A = torch.randn((m, n), generator=gen, device="cuda", dtype=dtype)
    B = torch.randn((n, p), generator=gen, device="cuda", dtype=dtype)
    C = torch.empty((m, p), device="cuda", dtype=dtype)
    flags = {"one": moa.MOA_FLAG_FP8_ONE_TERM, "two": moa.MOA_FLAG_FP8_TWO_TERM}.get(fp8, 0)
    d = moa.make_desc(A, B, C, path=path, flags=flags)
    L, st = moa.lib(), torch.cuda.current_stream().cuda_stream

    def f():
        if L.moa_gemm(ctypes.byref(d), st) != 0:
            raise RuntimeError(moa.moa_last_error())
    for _ in range(args.warmup):
        f()
    per, tot = timed_loop(f, args.steps, torch)
    if args.copy_calibration:
        src = torch.empty(COPY_CAL_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps({"profile_case": name, "m": m, "n": n, "p": p, "dtype": dt, "plan": moa.moa_plan_query(d),
                      "launches": args.steps, "ms_per_launch": round(tot / args.steps, 4),
                      "per_launch_ms": [round(x, 4) for x in per],
                      "tflops": round(2.0 * m * n * p / (tot / args.steps) / 1e9, 2)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2306_11148_amd import inputs, moa

    moa.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile_case:
        profile_case(args, torch, moa)
        return
    if args.sweep:
        sweep(args, torch, moa, inputs)
        return
    if args.block_sweep:
        block_sweep(args, torch, moa)
        return
    if args.split_variants:
        split_variants(args, torch, moa)
        return
    if args.split_k:
        split_k_sweep(args, torch, moa, inputs)
        return
    if args.layouts:
        layout_sweep(args, torch, moa)
        return
    if args.ipophp:
        ipophp_section(torch, moa)
        return
    if args.serve_rates:
        for rate in [float(x) for x in args.serve_rates.split(",")]:
            progress(f"serving loop at {rate:.0f} req/s: up to {args.serve_seconds:.1f} s or "
                     f"{args.serve_requests} requests")
            res, kept = serving_section(torch, moa, inputs, rate, args.serve_seconds, args.serve_requests,
                                        window_us=args.serve_window, max_group=args.serve_max_group)
            res["verified"] = cpu_verify_serving(kept)
            print(json.dumps({"serving_sweep": res}), flush=True)
        return
    N = args.n
    A_h, B_h = inputs.normal_f32(N, N, N, seed=N)
    A = torch.from_numpy(A_h).to(dev)
    B = torch.from_numpy(B_h).to(dev)
    C = torch.empty((N, N), dtype=torch.float32, device=dev)
    C_onf = torch.empty_like(C)
    desc_split = moa.make_desc(A, B, C, path=moa.MOA_PATH_SPLIT_BF16)
    desc_onf = moa.make_desc(A, B, C_onf, path=moa.MOA_PATH_ONF)
    plan_split = moa.moa_plan_query(desc_split)
    plan_onf = moa.moa_plan_query(desc_onf)
    stream = torch.cuda.current_stream().cuda_stream
    L = moa.lib()
    import ctypes
    pd_split, pd_onf = ctypes.byref(desc_split), ctypes.byref(desc_onf)

    def step():
        s = L.moa_gemm(pd_split, stream)
        if s != 0:
            raise RuntimeError(moa.moa_last_error())

    def onf():
        s = L.moa_gemm(pd_onf, stream)
        if s != 0:
            raise RuntimeError(moa.moa_last_error())

    progress(f"split-BF16 N={N}: {args.warmup} warm-up + {args.steps} timed steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    per, total_ms = timed_loop(step, args.steps, torch)
    ms = total_ms / args.steps
    # the same loop again with the library's event tracing on: per-kernel
    # times of the contraction and of the operand conditioning
    moa.moa_trace_read(reset=True)
    moa.moa_trace_enable(True)
    timed_loop(step, args.steps, torch)
    moa.moa_trace_enable(False)
    traced = moa.moa_trace_read(reset=True)
    n_k, ms_k = traced.get("split_bf16", (0, 0.0))
    kernel_ms = ms_k / n_k if n_k else ms
    n_p, ms_p = traced.get("split_pack", (0, 0.0))
    pack_ms = ms_p / n_p if n_p else None
    flops = 2.0 * N ** 3
    tflops = flops / (ms * 1e-3) / 1e12
    issued = 3 * flops / (ms * 1e-3) / 1e12
    issued_kernel = 3 * flops / (kernel_ms * 1e-3) / 1e12

    progress(f"ONF N={N}: {args.onf_steps} timed steps")
    onf()
    per_onf, total_onf = timed_loop(onf, args.onf_steps, torch)
    ms_onf = total_onf / args.onf_steps
    tflops_onf = flops / (ms_onf * 1e-3) / 1e12

    if not args.no_energy:
        progress("energy per call (split-BF16, ONF)")
    energy = None if args.no_energy else Energy()
    e_split = energy_per_call(step, args.energy_seconds, ms, energy, torch)
    e_onf = energy_per_call(onf, args.energy_seconds, ms_onf, energy, torch)

    if args.copy_calibration:
        # one device-to-device copy of exactly COPY_CAL_BYTES, identifiable by size
        src = torch.empty(COPY_CAL_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    progress(f"FP64 ONF N={N} and 256^3")
    fp64, fp64_keep = fp64_sections(torch, moa, inputs, N, max(3, args.onf_steps // 2), energy)

    if not args.no_grouped:
        progress("grouped products")
    grouped = None if args.no_grouped else grouped_section(torch, moa, inputs)
    if not args.no_precision:
        progress("precision workload")
    precision, precision_keep = (None, None) if args.no_precision else precision_section(torch, moa, inputs)
    if not args.no_serving:
        progress("serving loop")
    serving, serving_kept = (None, None) if args.no_serving else serving_section(
        torch, moa, inputs, args.serve_rate, args.serve_seconds, args.serve_requests)

    C_h = C.cpu().numpy()
    onf_h = C_onf.cpu().numpy()
    cpu = None
    err_split = err_onf = None
    if not args.no_cpu_baseline:
        progress(f"CPU oracle baseline (about {args.cpu_seconds:.0f} s)")
        onf_rows = np.arange(0, N, max(1, N // 64))
        cpu, errs = cpu_baseline(A_h, B_h, C_h, N, args.cpu_seconds, (onf_rows, onf_h[onf_rows]),
                                 precision_keep)
        err_split, err_onf = errs["split_bf16"], errs.get("onf_f32")
        e64 = cpu_check_fp64(fp64_keep)
        fp64["onf_f64"]["normwise_err_sampled"] = e64["onf_f64_sampled"]
        fp64["c1_256_f64"]["normwise_err"] = e64["c1"]
        fp64["c1_256_f64"]["integer_bitwise"] = e64["c1_integer_bitwise"]
        if serving is not None:
            progress("CPU check of the sampled served results")
            serving["verified"] = cpu_verify_serving(serving_kept)
        if precision is not None and "precision" in errs:
            for k, (e, er) in errs["precision"].items():
                precision[k]["normwise_err"] = e
                precision[k]["max_row_rel_err"] = er

    result = {
        "metric": "TFLOP/s + % peak at N=8192 (ONF vs split-BF16 MFMA); p50/p99 GEMM latency",
        "value": round(tflops, 2),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic: A, B i.i.d. N(0,1) FP32, numpy PCG64 seed N",
        "config": {"workload": f"square FP32 product m=n=p={N}, split-BF16 matrix-core path "
                               "(3 BF16 products, FP32 accumulate)",
                   "N": N, "in_out_dtype": "f32", "plan": plan_split},
        "pct_of_bf16_peak_issued": round(100 * issued / BF16_PEAK_TF, 2),
        "latency_ms": {"p50": round(pct(per, 50), 4), "p99": round(pct(per, 99), 4),
                       "min": round(min(per), 4), "max": round(max(per), 4)},
        "roofline": {"bound": "mfma", "achieved": round(issued_kernel, 2), "peak": BF16_PEAK_TF,
                     "unit": "TFLOP/s", "frac": round(issued_kernel / BF16_PEAK_TF, 4),
                     "traffic": measured_traffic(SPLIT_KERNEL_SOURCES, "profiles/split_bf16_N8192_traffic.json")
                     if N == 8192 else None,
                     "kernel": "ring::single_kernel<256, 256, 128, 64, 1, SplitMode, 3> (split-BF16 contraction)",
                     "work_per_launch": "3 * 2 N^3 BF16 matrix-core flop (hi.hi + hi.lo + lo.hi)",
                     "avg_kernel_ms": round(kernel_ms, 4),
                     "kernel_timing": "HIP events on the launch stream (library tracing)",
                     "conditioning_kernels_ms": None if pack_ms is None else round(pack_ms, 4)},
        "onf": {"tflops": round(tflops_onf, 2), "ms": round(ms_onf, 3),
                "roofline": {"bound": "alu", "achieved": round(tflops_onf, 2), "peak": FP32_VEC_PEAK_TF,
                             "unit": "TFLOP/s", "frac": round(tflops_onf / FP32_VEC_PEAK_TF, 4)},
                "p50_ms": round(pct(per_onf, 50), 3), "p99_ms": round(pct(per_onf, 99), 3),
                "plan": plan_onf, "normwise_err_sampled": err_onf},
        "split_speedup_over_onf": round(ms_onf / ms, 3),
        "normwise_err_split_sampled": err_split,
        "energy": {"split_bf16": e_split, "onf": e_onf,
                   "note": None if (energy and energy.h is not None) else
                   (energy.err if energy else "disabled")},
        "fp64": fp64,
        "grouped": grouped,
        "serving": serving,
        "precision": precision,
        "cpu_baseline": cpu,
    }
    clk = (e_split or {}).get("median_gfx_clock_mhz")
    if clk:
        # the board's power cap holds the clock below 2.4 GHz under this load:
        # the same kernel time against the peak scaled to the sampled clock
        result["roofline"]["gfx_clock_mhz_sampled"] = clk
        result["roofline"]["frac_of_clock_scaled_peak"] = round(issued_kernel / (BF16_PEAK_TF * clk / 2400.0), 4)
    if e_split and e_onf:
        result["energy"]["onf_over_split_joules"] = round(
            e_onf["joules_per_gemm"] / e_split["joules_per_gemm"], 3)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
