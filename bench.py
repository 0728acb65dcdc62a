#!/usr/bin/env python3
"""Benchmark of the MoA ONF matrix product on one MI355X.

Workload: C = A.B with m = n = p = 8192, FP32 row-major operands drawn
i.i.d. N(0, 1) (seeded, synthetic), resident in HBM before timing starts.

One step = one product on the split-BF16 matrix-core path (operand split
fused into LDS staging, three BF16 products per fragment, FP32 accumulation,
epilogue store): the whole path for one input. `value` is effective TFLOP/s
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
FP32_VEC_PEAK_TF = 157.3    # FP32 vector peak with packed FMA, MI355X
FP32_FMA_UNPACKED_TF = 78.6  # one v_fma_f32 per lane per clock: 256 CU x 64 lanes x 2 x 2.4 GHz
FP8_PEAK_TF = 5033.2


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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of known size (for counter scaling)")
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


def measured_traffic(kernel_source: str, record: str):
    """HBM bytes per launch from the committed counter record, or None when the
    kernel source has changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, record)))
        sha = hashlib.sha256(open(os.path.join(ROOT, kernel_source), "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


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
    if energy is None or energy.h is None:
        return None
    reps = max(5, int(seconds * 1e3 / max(ms_each, 1e-3)))
    torch.cuda.synchronize()
    e0, t0 = energy.joules(), time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    e1, t1 = energy.joules(), time.perf_counter()
    snap = energy.snapshot()
    return {"joules_per_gemm": (e1 - e0) / reps, "reps": reps, "seconds": t1 - t0,
            "avg_power_w": (e1 - e0) / (t1 - t0), **snap}


def cpu_baseline(A, B, C_gpu, n, target_s):
    """The FP64 oracle on a seeded row sample of the same product."""
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
    err = O.rel_err(C_gpu[all_rows], Rall)
    return {"value": flops / done_t / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(all_rows)} seeded rows of the {n}^3 FP32 product (inputs widened to "
                      f"FP64), {done_t:.1f} s of oracle time",
            "seconds": done_t}, err


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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    per, total_ms = timed_loop(step, args.steps, torch)
    ms = total_ms / args.steps
    flops = 2.0 * N ** 3
    tflops = flops / (ms * 1e-3) / 1e12
    issued = 3 * flops / (ms * 1e-3) / 1e12

    onf()
    per_onf, total_onf = timed_loop(onf, args.onf_steps, torch)
    ms_onf = total_onf / args.onf_steps
    tflops_onf = flops / (ms_onf * 1e-3) / 1e12

    energy = None if args.no_energy else Energy()
    e_split = energy_per_call(step, args.energy_seconds, ms, energy, torch)
    e_onf = energy_per_call(onf, args.energy_seconds, ms_onf, energy, torch)

    if args.copy_calibration:
        src = torch.empty(256 * 2 ** 20 // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    C_h = C.cpu().numpy()
    onf_h = C_onf.cpu().numpy()
    cpu = None
    err_split = err_onf = None
    if not args.no_cpu_baseline:
        cpu, err_split = cpu_baseline(A_h, B_h, C_h, N, args.cpu_seconds)
        from oracle import oracle as O
        rows = np.arange(0, N, max(1, N // 64))
        Rs = O.gemm_rows_f64(A_h, B_h, rows)
        err_onf = O.rel_err(onf_h[rows], Rs)

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
        "roofline": {"bound": "mfma", "achieved": round(issued, 2), "peak": BF16_PEAK_TF,
                     "unit": "TFLOP/s", "frac": round(issued / BF16_PEAK_TF, 4),
                     "traffic": measured_traffic("paper_2306_11148_amd/csrc/split_bf16.hip",
                                                 "profiles/split_bf16_N8192_traffic.json")
                     if N == 8192 else None,
                     "kernel": "split_bf16_kernel",
                     "work_per_launch": "3 * 2 N^3 BF16 matrix-core flop (hi.hi + hi.lo + lo.hi)",
                     "avg_kernel_ms": round(ms, 4)},
        "onf": {"tflops": round(tflops_onf, 2), "ms": round(ms_onf, 3),
                "pct_of_fp32_vector_peak": round(100 * tflops_onf / FP32_VEC_PEAK_TF, 2),
                "pct_of_unpacked_fma_peak": round(100 * tflops_onf / FP32_FMA_UNPACKED_TF, 2),
                "p50_ms": round(pct(per_onf, 50), 3), "p99_ms": round(pct(per_onf, 99), 3),
                "plan": plan_onf, "normwise_err_sampled": err_onf},
        "split_speedup_over_onf": round(ms_onf / ms, 3),
        "normwise_err_split_sampled": err_split,
        "energy": {"split_bf16": e_split, "onf": e_onf,
                   "note": None if (energy and energy.h is not None) else
                   (energy.err if energy else "disabled")},
        "cpu_baseline": cpu,
    }
    if e_split and e_onf:
        result["energy"]["onf_over_split_joules"] = round(
            e_onf["joules_per_gemm"] / e_split["joules_per_gemm"], 3)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
