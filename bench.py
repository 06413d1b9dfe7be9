#!/usr/bin/env python3
"""LLOID filtering throughput on one MI355X: template SNR-samples per second.

A step is one 1-s stride of the whole path (decimation, basis correlation,
split reduction, mixing + upsample-and-add + series write, triggers) for
every template and detector of the workload, with the strain already
resident in device memory.  Prints one JSON line.

Workloads (synthetic, seeded; see synth/):
  realistic  1 detector, 1024 chirp templates, 5 rates 4096..256 Hz,
             L = 40/60/80/100/120, strain 4096 s at 4096 Hz (default)
  plain      1 detector, 64 templates, 2 rates (2048/512 Hz), 32 s
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "template SNR-samples/sec per MI355X, batched BF16 vs plain FP32 at SNR err≤1e-3"
PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0, "fp16": 2500.0, "fp8_bf16": 5000.0}
HBM_GBS = 8000.0


def workload(name: str):
    import synth
    if name == "realistic":
        return synth.cached_workload("c2", synth.config2)
    if name == "plain":
        return synth.config1()
    raise SystemExit(f"unknown workload {name}")


def kernel_flops(w, n_det: int) -> dict:
    """Algorithmic flops per launch of the two contraction kernels."""
    corr = mix = 0.0
    for bank in w.banks:
        M = bank.n_templates
        for s in bank.slices:
            corr += 2.0 * s.n_basis * s.n_taps * s.rate
            mix += 2.0 * (2 * M) * s.n_basis * s.rate
        rates = sorted({s.rate for s in bank.slices} | {w.sample_rate}, reverse=True)
        for hi, lo in zip(rates[:-1], rates[1:]):
            mix += 2.0 * (2 * M) * (hi - lo) * 17
    return {"corr": corr * n_det, "mix": mix * n_det}


def cpu_baseline(w, x, first: int, seconds: float, gpu_series=None):
    """The FP64 oracle on the host cores for a bounded sample of strides."""
    import numpy as np
    from oracle import lloid as O
    cores = len(os.sched_getaffinity(0))
    cfg = O.OracleConfig(w.sample_rate)
    F = w.sample_rate
    done, t0 = 0, time.perf_counter()
    refs = []
    while True:
        k = first + done
        z, _ = O.lloid_filter(x[0, :(k + 1) * F], w.banks[0], cfg, n_strides=1, first_stride=k)
        refs.append(z)
        done += 1
        el = time.perf_counter() - t0
        if el >= seconds or done >= 64:
            break
    rate = w.n_templates * F * w.n_detectors * done / el
    out = {"value": rate, "unit": "SNR-samples/s", "cores": cores, "kind": "oracle",
           "sample": f"{done} strides ({done} s) from stride {first} of the same workload, float64 NumPy, "
                     f"BLAS threads = {cores}"}
    err = None
    if gpu_series is not None:
        zr = np.concatenate(refs, axis=1)
        n = min(zr.shape[1], gpu_series.shape[1])
        zr, zg = zr[:, :n], gpu_series[:, :n]
        err = float((np.abs(zg - zr) / np.maximum(np.abs(zr), 4.0)).max())
    return out, err, done


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2048)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--workload", default="realistic")
    ap.add_argument("--precision", default="fp32", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--peaks-only", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU: the filtering path has no multi-GPU "
                                   "form; run with --gpus 1"}))
        return 2

    import numpy as np
    import torch
    import synth
    from paper_2511_04730_amd import LloidPlan

    w = workload(args.workload)
    F, ND = w.sample_rate, w.n_detectors
    n_total = args.warmup + args.steps
    n_avail = w.duration_s
    x = synth.workload_strain(w, min(n_total, n_avail))
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    strides = [xs[:, (k % n_avail) * F:((k % n_avail) + 1) * F].contiguous() for k in range(min(n_total, n_avail))]

    plan = LloidPlan(w.banks, F, ND, args.precision)
    write = not args.peaks_only
    series = plan.new_series() if write else None
    peaks = plan.new_peaks()
    for k in range(args.warmup):
        plan.push(strides[k % len(strides)], series=series, peaks=peaks, write_series=write)
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} strides done", file=sys.stderr, flush=True)

    # timed region: K strides, per-kernel HIP events on the launch stream
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    for k in range(args.warmup, n_total):
        plan.push(strides[k % len(strides)], series=series, peaks=peaks, write_series=write)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    prof = plan.profile_read()
    plan.profile(False)
    print(f"[bench] timed {args.steps} strides: {ms:.2f} ms (wall {wall * 1e3:.2f} ms)", file=sys.stderr, flush=True)

    samples = w.n_templates * F * ND * args.steps
    value = samples / (ms / 1e3)
    kf = kernel_flops(w, ND)
    dom = max(("corr", "mix"), key=lambda k: prof[k][0])
    avg_ms = prof[dom][0] / max(prof[dom][1], 1)
    achieved = kf[dom] / (avg_ms / 1e3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    kernel_ms = {k: round(v[0] / max(v[1], 1), 5) for k, v in prof.items()}

    # parity sample + CPU baseline: rerun from zero history up to the sample
    base, err = None, None
    if not args.no_cpu_baseline and w.n_detectors == 1:
        first = min(64, len(strides) - 8)
        plan.reset()
        zs = []
        series2 = plan.new_series()
        for k in range(first + 8):
            plan.push(strides[k], series=series2, peaks=peaks, write_series=True)
            if k >= first:
                zs.append(plan.bank_view(series2, 0)[0].cpu().numpy().astype(np.complex128))
        torch.cuda.synchronize()
        base, err, n_cpu = cpu_baseline(w, x, first, args.cpu_seconds, np.concatenate(zs, axis=1))

    out = {
        "metric": METRIC, "value": value, "unit": "SNR-samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "bf16x3": "bf16x3", "fp16": "f16", "fp8_bf16": "fp8"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "templates": w.n_templates, "detectors": ND,
                   "rates_hz": sorted({s.rate for b in w.banks for s in b.slices}, reverse=True),
                   "precision": args.precision, "series_written": write, "stride_s": 1,
                   "flops_per_stride": plan.flops_per_stride},
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None},
        "kernel_ms": kernel_ms,
        "snr_err": err,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
