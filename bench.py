#!/usr/bin/env python3
"""LLOID filtering throughput on one MI355X: template SNR-samples per second.

A step is one 1-s stride of the whole path (decimation, basis correlation,
split reduction, mixing + upsample-and-add + series write, triggers) for
every template and detector of the workload, with the strain already
resident in device memory.  Prints one JSON line.

Workloads (synthetic, seeded; see synth/):
  batched    2 detectors, 200 uneven sub-banks (~120k templates, 3-7 rates
             4096..64 Hz, L 20-150, filters 0.5-64 s), 4096 Hz   (default)
  realistic  1 detector, 1024 chirp templates, 5 rates 4096..256 Hz,
             L = 40/60/80/100/120
  plain      1 detector, 64 templates, 2 rates (2048/512 Hz)
  largest    2 detectors, 800 uneven sub-banks (~474k templates, 3-6 rates
             4096..128 Hz, filters 0.5-128 s, N up to 97k), 4096 Hz; meant
             for --precision fp8_bf16

The default precision is bf16x3 (BF16 operands, both sides split, FP32
accumulation); --compare fp32 also times the plain FP32 path on the same
workload.  The SNR error against the FP64 oracle is measured on a sample of
banks at one stride in the same run.
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
HBM_GBS = 8000.0   # MI355X HBM3E peak
COINC_OVERLAP_S = 0.0273 + 0.005   # H-L-V light travel time + coincidence buffer


def kernel_peak(precision: str, kernel: str) -> float:
    """Dense MFMA peak of the arithmetic a kernel runs in: the FP8 form
    correlates in FP8 but mixes in BF16x3."""
    if precision == "fp8_bf16" and kernel == "mix":
        return PEAK_TFLOPS["bf16x3"]
    return PEAK_TFLOPS[precision]
DTYPE = {"fp32": "f32", "bf16x3": "bf16x3", "fp16": "f16x2", "fp8_bf16": "fp8"}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name: str):
    import synth
    if name == "largest":
        # ~11 GB of float64 bank: generated in memory each run, not cached
        return synth.config5(progress=log)
    if name == "batched":
        return synth.cached_workload("c3", synth.config3)
    if name == "realistic":
        return synth.cached_workload("c2", synth.config2)
    if name == "plain":
        return synth.config1()
    raise SystemExit(f"unknown workload {name}")


KERNEL_SOURCES = {"mix": ["lloid_mix.hip", "lloid_internal.h", "lloid_device.h", "lloid_mfma.h"],
                  "corr": ["lloid_corr.hip", "lloid_internal.h", "lloid_device.h", "lloid_mfma.h"],
                  "xi2": ["lloid_xi2.hip", "lloid_xi2.h", "lloid_internal.h", "lloid_device.h"],
                  "window_trigger": ["lloid_coinc.hip", "lloid_coinc.h", "lloid_internal.h", "lloid_device.h"],
                  "whitening": ["lloid_whiten.hip", "lloid_whiten.h"],
                  "down": ["lloid_kernels.hip", "lloid_internal.h", "lloid_device.h"],
                  "peaks": ["lloid_kernels.hip", "lloid_internal.h", "lloid_device.h"]}


def source_digest(kernel: str) -> str:
    """sha256 over the sources a kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2511_04730_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/traffic_counters.txt (lines: kernel/workload/precision,
    bytes per launch, source sha256; '#' lines give the commands), i.e.
    FETCH_SIZE and WRITE_SIZE per dispatch scaled by the copy-kernel
    calibration; None when there is no entry or the kernel's sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 3 and not line.startswith("#") and parts[0] == f"{kernel}/{workload}/{precision}":
                return float(parts[1]) if parts[2] == source_digest(kernel) else None
    return None


def kernel_flops(w) -> dict:
    """Algorithmic flops per launch of the two contraction kernels (all
    banks and detectors)."""
    corr = mix = 0.0
    for bank in w.banks:
        M = bank.n_templates
        for s in bank.slices:
            corr += 2.0 * s.n_basis * s.n_taps * s.rate
            mix += 2.0 * (2 * M) * s.n_basis * s.rate
        rates = sorted({s.rate for s in bank.slices} | {w.sample_rate}, reverse=True)
        for hi, lo in zip(rates[:-1], rates[1:]):
            mix += 2.0 * (2 * M) * (hi - lo) * 17
    return {"corr": corr * w.n_detectors, "mix": mix * w.n_detectors}


ELT_U = {"fp32": 4, "bf16x3": 4, "fp16": 2, "fp8_bf16": 1}    # bytes per basis value (hi + lo where split)
ELT_W = {"fp32": 4, "bf16x3": 4, "fp16": 2, "fp8_bf16": 4}    # bytes per mixing value (FP8 form mixes in BF16x3)
MIX_TN = 256                                                   # top-rate samples per mixing time tile


def kernel_bytes(w, precision: str, write_series: bool = True) -> dict:
    """Algorithmic HBM bytes per launch of the stride's kernels (all banks and
    detectors): what each kernel must read or write at least once.
      down   the stride's strain read, every decimated stream written (4 B)
      corr   every basis read once, every new basis output written (4 B:
             FP32 or the hi + lo halves)
      mix    every mixing row read once, every detector's basis-output window
             read once, the SNR series written (8 B per SNR-sample), one
             16-B trigger candidate per template, detector and time tile
      peaks  the candidates read, one 20-B trigger per template and detector"""
    nd, F = w.n_detectors, w.sample_rate
    ntt = F // MIX_TN
    out = {"down": 0.0, "corr": 0.0, "mix": 0.0, "peaks": 0.0}
    rates = set()
    for bank in w.banks:
        M = bank.n_templates
        for s in bank.slices:
            rates.add(s.rate)
            y = 4.0 * s.n_basis * s.rate * nd
            out["corr"] += ELT_U[precision] * s.n_basis * s.n_taps + y
            out["mix"] += ELT_W[precision] * 2 * M * s.n_basis + y
        out["mix"] += nd * M * ((8.0 * F if write_series else 0.0) + 16.0 * ntt)
        out["peaks"] += nd * M * (16.0 * ntt + 20.0)
    out["down"] = nd * 4.0 * (F + sum(r for r in rates if r < F))
    return out


def roof(flops: float, nbytes: float, ms: float, mfma_peak_tflops: float) -> dict:
    """Both roofs of one kernel: the fraction of the MFMA peak its
    algorithmic flops reach and of the HBM peak its algorithmic bytes reach
    in `ms`; `bound` is the roof with the larger ideal time, `frac` its
    fraction."""
    t_mfma = flops / (mfma_peak_tflops * 1e12) if flops else 0.0
    t_hbm = nbytes / (HBM_GBS * 1e9)
    sec = ms / 1e3
    r = {"ms": ms, "flops": flops, "bytes": nbytes,
         "mfma_tflops": flops / sec / 1e12, "mfma_peak": mfma_peak_tflops, "mfma_frac": t_mfma / sec,
         "hbm_gbs": nbytes / sec / 1e9, "hbm_peak": HBM_GBS, "hbm_frac": t_hbm / sec}
    r["bound"] = "mfma" if t_mfma > t_hbm else "hbm"
    r["frac"] = max(t_mfma, t_hbm) / sec
    return r


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed(plan, strides, warmup: int, steps: int, write: bool, profile: bool):
    import torch
    series = plan.new_series() if write else None
    peaks = plan.new_peaks()
    n = len(strides)
    for k in range(warmup):
        plan.push(strides[k % n], series=series, peaks=peaks, write_series=write)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if profile:
        plan.profile(True)
    torch.cuda.synchronize()
    e0.record(st)
    for k in range(warmup, warmup + steps):
        plan.push(strides[k % n], series=series, peaks=peaks, write_series=write)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = plan.profile_read() if profile else None
    if profile:
        plan.profile(False)
    del series, peaks
    return ms, prof


def downstream_measure(plan, w, strides, reps: int):
    """The consumers of the SNR series on strides 0..2 of every bank and
    detector, each timed over `reps` launches with HIP events:
    xi^2 (Sec. II.D.2) at the triggers of stride 1 with seeded chirp-like
    autocorrelations of 351 or 701 samples per bank (algorithmic bytes: per
    trigger the A-sample complex window, the trigger and the output; per
    template its autocorrelation), and the overlapping trigger windows plus
    coincidence and clustering (Sec. II.D.3-4) of stride 2 with the H-L-V
    overlap of 0.0323 s (window triggers: per trigger the overlap's complex
    samples, the stride trigger read and the window trigger written)."""
    import numpy as np
    import torch
    import synth
    lengths = [synth.acf_length(b) for b in w.banks]
    parts = []
    for b, (bank, A) in enumerate(zip(w.banks, lengths)):
        R = synth.synthetic_acf(w.config, b, bank.n_templates, A)
        parts.append(np.stack([R.real, R.imag], axis=-1).reshape(-1))
    acf = torch.from_numpy(np.concatenate(parts)).cuda()
    del parts
    plan.set_autocorrelation(acf, lengths)
    del acf
    plan.reset()
    ser = [plan.new_series() for _ in range(3)]
    pk = [plan.new_peaks() for _ in range(3)]
    for k in range(3):
        plan.push(strides[k], series=ser[k], peaks=pk[k])
    out = torch.empty(plan.n_peaks, dtype=torch.float32, device="cuda")
    nd = w.n_detectors
    ov = int(round(COINC_OVERLAP_S * w.sample_rate))
    win = np.full((nd, nd), ov)
    trig, ev = plan.coincidence(pk[2], win, ov, prev=ser[1])
    plan.xi2(ser[1], pk[1], prev=ser[0], next=ser[2], out=out)
    torch.cuda.synchronize()
    plan.profile(True)
    for _ in range(reps):
        plan.xi2(ser[1], pk[1], prev=ser[0], next=ser[2], out=out)
    for _ in range(reps):
        plan.coincidence(pk[2], win, ov, prev=ser[1], triggers=trig, events=ev)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    ms, n = prof["xi2"]
    finite = bool(torch.isfinite(out).all().item())
    n_events = sum(1 for e in plan.events_view(ev) if e[0] >= 0)
    del ser, pk, out, trig, ev
    byt = sum(nd * b.n_templates * (8 * A + 20 + 4) + b.n_templates * 8 * A for b, A in zip(w.banks, lengths))
    n_trig = nd * w.n_templates
    return {"ms": ms / max(n, 1), "launches": n, "bytes": byt, "finite": finite,
            "acf_lengths": {str(a): lengths.count(a) for a in sorted(set(lengths))},
            "trig_ms": prof["triggers"][0] / max(prof["triggers"][1], 1),
            "coinc_ms": prof["coinc"][0] / max(prof["coinc"][1], 1),
            "trig_bytes": n_trig * (8 * ov + 20 + 20), "events": n_events, "overlap": ov}


WHITEN_RATE_IN = 16384   # strain rate the whitener reads (Hz)


def whiten_measure(w, reps: int):
    """Whitening with frequency-domain downsampling (Sec. II.B.2) at the
    paper's low-latency setting: 4 s blocks of 16384 Hz strain with 1 s of
    zero padding (one push per second), output at the workload's top rate,
    median of 7, for every detector.  Returns the mean HIP-event time of one
    push over `reps` pushes after 8 untimed ones, and its algorithmic bytes
    per detector: the new hop of strain and the block read once, the PSD's
    median ring read and its new entry written (n_med + 1 values per output
    bin), the PSD estimate written, the overlap-add state read and written
    and the output hop written.  The FFT passes' intermediate traffic is not
    counted: it is what this implementation adds, not what the method needs
    (the push is bound by the latency of its launches, one per pass)."""
    import math
    import numpy as np
    import torch
    from paper_2511_04730_amd import Whitener
    N, Z, D = 4 * WHITEN_RATE_IN, WHITEN_RATE_IN, WHITEN_RATE_IN // w.sample_rate
    nd = w.n_detectors
    wh = Whitener(nd, N, Z, D)
    g = np.random.default_rng([w.config, 7, 0])
    xs = [torch.from_numpy(g.standard_normal((nd, wh.hop)).astype(np.float32)).cuda() for _ in range(4)]
    out = torch.empty((nd, wh.hop_out), dtype=torch.float32, device="cuda")
    for i in range(8):
        wh.push(xs[i % 4], out=out)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for i in range(reps):
        wh.push(xs[i % 4], out=out)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    finite = bool(torch.isfinite(out).all().item())
    n_out, K, H = N // D, N // D // 2 + 1, wh.hop
    passes = lambda n: (int(math.log2(n)) + 1) // 2      # radix-4 passes (one radix-2 pass if log2 n is odd)
    per_det = 4 * H + 4 * N + K * 4 * (7 + 1) + 8 * K + 8 * n_out + 4 * (H // D)
    launches = 3 + passes(N) + passes(n_out)
    wh.close()
    return {"ms_per_push": ms, "block": N, "pad": Z, "decimation": D, "rate_in_hz": WHITEN_RATE_IN,
            "launches_per_push": launches, "bytes": per_det * nd, "finite": finite}


def svd_measure(reps: int = 3, rows: int = 2048, n: int = 1024, rank: int = 40, iters: int = 30):
    """SVD bank construction (Sec. II.C.1) for one slice of the realistic
    bank's shape (2M = 2048 real templates, N = 1024 taps, L = 40): a seeded
    matrix with the spectrum 0.8^k, `iters` subspace iterations, mean wall
    time over `reps` calls (each synchronises), and the residual
    ||H - W U||_F over the optimum.  Algorithmic flops per call: iters x (2
    products of 2 rows N L + one CholeskyQR pass on each half step, 2 L^2
    rows and 2 L^2 N, + 2 L^3 / 3) + the final product."""
    import numpy as np
    import torch
    from paper_2511_04730_amd.plan import svd_basis
    g = np.random.default_rng([42, 11, 0])
    A = np.linalg.qr(g.standard_normal((rows, rank * 2)))[0]
    B = np.linalg.qr(g.standard_normal((n, rank * 2)))[0]
    H = torch.from_numpy((A * 0.8 ** np.arange(rank * 2)) @ B.T).cuda()
    start = torch.from_numpy(g.standard_normal((rank, n))).cuda()
    U, W = svd_basis(H, rank, start, iters=iters)
    torch.cuda.synchronize()
    # residual against the optimum: the spectrum is 0.8^k by construction,
    # so the best rank-L residual is sqrt(sum_{k >= L} 0.8^(2k))
    resid = float(torch.linalg.norm(H - W @ U))
    opt = float(np.sqrt(np.sum(0.8 ** (2 * np.arange(rank, 2 * rank)))))
    t0 = time.perf_counter()
    for _ in range(reps):
        svd_basis(H, rank, start, iters=iters)
    ms = (time.perf_counter() - t0) / reps * 1e3
    flops = iters * (4 * rows * n * rank + 2 * rank * rank * (rows + n) + 2 * rank ** 3 / 3) + 2 * rows * n * rank
    return {"ms": ms, "rows": rows, "taps": n, "rank": rank, "iterations": iters,
            "residual_over_optimum": resid / opt,
            "roofline": {"bound": "mfma", "achieved": flops / (ms / 1e3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                         "frac": flops / (ms / 1e3) / 1e12 / 78.6, "dtype": "f64",
                         "limited_by": "latency of the per-step factorisation and launches"}}


def grad_measure(reps: int = 3, refine_steps: int = 0, tune: bool = False):
    """The gradient workload: the realistic bank (1024 templates, 5 rates)
    at half its basis counts (L = 20/30/40/50/60), 64 s of strain at
    4096 Hz, target = the FP32 output of the same bank at its full basis
    counts.  Times lloid_grad (forward over the 64 strides with capture,
    residual, transposed chain and the dW / dU contractions, synchronised)
    as the mean of `reps` calls after one untimed, and optionally
    `refine_steps` steps of refinement with FP64 re-orthonormalisation.
    With `tune`, the FP32 plan's tiling is autotuned on the segment's first
    four strides first (the forward strides inside the gradient use it)."""
    import numpy as np
    import torch
    import synth
    from paper_2511_04730_amd import LloidPlan
    F, T = 4096, 64
    full = synth.config2(duration_s=T).banks[0]
    half = synth.truncate_bank(full, synth.C4_BASIS)
    x = torch.from_numpy(synth.gaussian_strain(4, 1, T * F).astype(np.float32)).cuda()
    tp = LloidPlan([full], F, 1, "fp32", normalize=False)
    tg = torch.empty((T, tp.series_floats), dtype=torch.float32, device="cuda")
    for k in range(T):
        tp.push(x[:, k * F:(k + 1) * F].contiguous(), series=tg[k])
    torch.cuda.synchronize()
    tp.close()
    plan = LloidPlan([half], F, 1, "fp32", normalize=False)
    keys = ("corr_cols", "corr_split", "corr_group", "mix_group", "mix_tblock")
    if tune:
        from paper_2511_04730_amd.autotune import autotune
        autotune(plan, [x[:, k * F:(k + 1) * F].contiguous() for k in range(4)])
    tiling = {k: plan.option(k) for k in keys}
    loss, _, _ = plan.grad(x, tg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.grad(x, tg)
    ms = (time.perf_counter() - t0) / reps * 1e3
    # forward flops of the segment and the backward's three contractions
    # (dW = 2 G Y^T and dY = 2 W^T G per slice at its rate, dU a correlation
    # of dY with the slice's stream)
    M = half.n_templates
    fwd = bwd = 0.0
    for s in half.slices:
        fwd += T * (2.0 * s.n_basis * s.n_taps * s.rate + 2.0 * 2 * M * s.n_basis * s.rate)
        bwd += T * (2 * 2.0 * 2 * M * s.n_basis * s.rate + 2.0 * s.n_basis * s.n_taps * s.rate)
    out = {"ms": ms, "templates": M, "seconds": T, "basis": [s.n_basis for s in half.slices], "loss": loss,
           "flops": fwd + bwd, "tflops": (fwd + bwd) / (ms / 1e3) / 1e12, "tiling": tiling}
    if refine_steps:
        from paper_2511_04730_amd.refine import refine
        smax2 = max(float(np.linalg.norm(s.mixing, 2)) ** 2 for s in half.slices)
        t0 = time.perf_counter()
        losses, _, _ = refine(plan, [half], x, tg, steps=refine_steps, eta=0.25, eta_u=0.1 / smax2)
        torch.cuda.synchronize()
        out["refine"] = {"steps": refine_steps, "seconds": time.perf_counter() - t0, "loss_first": losses[0],
                         "loss_last": losses[-1],
                         "monotone": all(b <= a * (1 + 1e-7) for a, b in zip(losses, losses[1:]))}
    plan.close()
    return out


def gpu_stride_series(plan, strides, k: int):
    """The plan's series of stride k (fresh run of strides 0..k), per bank
    and detector 0, as complex128 host arrays."""
    import numpy as np
    import torch
    plan.reset()
    series = plan.new_series()
    peaks = plan.new_peaks()
    for i in range(k + 1):
        plan.push(strides[i], series=series, peaks=peaks, write_series=(i == k))
    torch.cuda.synchronize()
    return series


def parity_and_baseline(plan, w, x, strides, k: int, seconds: float, repeats: int = 5):
    """The oracle (FP64 NumPy on the host cores) on detector 0 for stride k
    of the first banks, as many as fill about seconds / (repeats + 2) per
    repeat; `repeats` timed repeats with all host threads (median) and the
    first bank alone with a single BLAS thread; the SNR error of the GPU series of the same
    banks and stride against it.  Returns (cpu_baseline dict, max SNR error,
    banks sampled)."""
    import numpy as np
    from oracle import lloid as O
    from threadpoolctl import threadpool_limits
    F = w.sample_rate
    series = gpu_stride_series(plan, strides, k)
    cfg = O.OracleConfig(F)
    cores = len(os.sched_getaffinity(0))
    xd = x[0, :(k + 1) * F]
    # first pass: choose the sample, check parity
    err, nb, samples, t0 = 0.0, 0, 0, time.perf_counter()
    budget = seconds / (repeats + 2)
    zs = []
    for b, bank in enumerate(w.banks):
        z, _ = O.lloid_filter(xd, bank, cfg, n_strides=1, first_stride=k)
        zs.append(z)
        samples += bank.n_templates * F
        nb += 1
        zg = plan.bank_view(series, b)[0].cpu().numpy().astype(np.complex128)
        err = max(err, float((np.abs(zg - z) / np.maximum(np.abs(z), 4.0)).max()))
        if time.perf_counter() - t0 >= budget:
            break
    del series

    def one_pass(n):
        ts = time.perf_counter()
        for bank in w.banks[:n]:
            O.lloid_filter(xd, bank, cfg, n_strides=1, first_stride=k)
        return time.perf_counter() - ts

    times = [one_pass(nb) for _ in range(repeats)]
    with threadpool_limits(1):
        t1 = one_pass(1)
    med = float(np.median(times))
    base = {"value": samples / med, "unit": "SNR-samples/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "repeats": repeats, "seconds_per_repeat": times,
            "value_1thread": w.banks[0].n_templates * F / t1,
            "sample": f"stride {k} of detector 0 for the first {nb} of {len(w.banks)} banks "
                      f"({samples} SNR-samples), float64 NumPy, BLAS threads = {cores} (median of {repeats} "
                      f"repeats); value_1thread: the first bank with one BLAS thread"}
    return base, err, zs


def leg_error(plan, strides, k: int, zs) -> float:
    """SNR error of another plan's stride-k series against the oracle series
    `zs` of the first len(zs) banks (detector 0)."""
    import numpy as np
    series = gpu_stride_series(plan, strides, k)
    err = 0.0
    for b, z in enumerate(zs):
        zg = plan.bank_view(series, b)[0].cpu().numpy().astype(np.complex128)
        err = max(err, float((np.abs(zg - z) / np.maximum(np.abs(z), 4.0)).max()))
    return err


def bank_loop(w, strides, warmup: int, steps: int, precision: str = "fp32"):
    """The unstacked baseline: one plan per bank, each filtering the stride
    with its own launches (no graph), banks in a host loop per stride.
    Returns ms for `steps` strides."""
    import torch
    from paper_2511_04730_amd import LloidPlan
    F, ND = w.sample_rate, w.n_detectors
    plans = [LloidPlan([b], F, ND, precision) for b in w.banks]
    outs = [(p.new_series(), p.new_peaks()) for p in plans]
    n = len(strides)
    for k in range(warmup):
        for p, (se, pk) in zip(plans, outs):
            p.push(strides[k % n], series=se, peaks=pk)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for k in range(warmup, warmup + steps):
        for p, (se, pk) in zip(plans, outs):
            p.push(strides[k % n], series=se, peaks=pk)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    for p in plans:
        p.close()
    del outs
    return ms


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="batched", choices=["batched", "realistic", "plain", "largest"])
    ap.add_argument("--precision", default="bf16x3", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--compare", default="fp32,fp16", help="also time these precisions, comma-separated ('' to skip)")
    ap.add_argument("--graph", type=int, default=1, help="replay one HIP graph per stride")
    ap.add_argument("--peaks-only", action="store_true", help="time without writing the series")
    ap.add_argument("--peaks-only-leg", type=int, default=1, help="also time the peaks-only mode")
    ap.add_argument("--loop-leg", type=int, default=-1,
                    help="also time one FP32 plan per bank in a host loop (-1: batched workload only)")
    ap.add_argument("--autotune", type=int, default=1, help="tune the tiling options before timing")
    ap.add_argument("--tiling", default="", help="fixed tiling instead of autotuning, "
                                                 "e.g. corr_split=8192,corr_group=32,mix_group=16")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--xi2", type=int, default=-1,
                    help="also time xi^2, coincidence, whitening and SVD construction (-1: all but the largest workload)")
    ap.add_argument("--grad-leg", type=int, default=0,
                    help="also time the gradient on the realistic bank at half rank (64 s)")
    ap.add_argument("--refine-steps", type=int, default=0, help="with --grad-leg: refinement steps to time")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU: the filtering path has no multi-GPU "
                                   "form; run with --gpus 1"}))
        return 2
    big = args.workload in ("batched", "largest")
    steps = args.steps if args.steps is not None else (32 if big else 2048)
    warmup = args.warmup if args.warmup is not None else (8 if big else 64)

    import numpy as np
    import torch
    import synth
    from paper_2511_04730_amd import LloidPlan

    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {n * 4} bytes read, {n * 4} bytes written")
        del src, dst

    w = workload(args.workload)
    F, ND = w.sample_rate, w.n_detectors
    k_par = min(64, w.duration_s - 1)
    n_str = min(max(warmup + steps, k_par + 1), w.duration_s)
    x = synth.workload_strain(w, n_str)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    strides = [xs[:, k * F:(k + 1) * F].contiguous() for k in range(n_str)]
    log(f"workload {w.name}: {w.n_templates} templates, {ND} det, {n_str} strides staged")
    write = not args.peaks_only
    kf = kernel_flops(w)

    tiling = {}

    def run(precision: str, profile: bool):
        plan = LloidPlan(w.banks, F, ND, precision)
        if args.tiling:
            for kv in args.tiling.split(","):
                k, v = kv.split("=")
                plan.set_option(k.strip(), int(v))
            tiling[precision] = {k: plan.option(k) for k in ("corr_cols", "corr_split", "corr_group", "mix_group", "mix_tblock")}
        elif args.autotune:
            from paper_2511_04730_amd.autotune import autotune
            best = autotune(plan, strides[:4], write_series=write, log=log)
            tiling[precision] = {k: best[k] for k in ("corr_cols", "corr_split", "corr_group", "mix_group", "mix_tblock")}
        else:
            tiling[precision] = {k: plan.option(k) for k in ("corr_cols", "corr_split", "corr_group", "mix_group", "mix_tblock")}
        if args.graph and not profile:
            plan.set_graph(True)
        ms, prof = timed(plan, strides, warmup, steps, write, profile)
        return plan, ms, prof

    plan, ms, _ = run(args.precision, profile=False)
    log(f"{args.precision}: {steps} strides in {ms:.2f} ms")
    samples = w.n_templates * F * ND * steps
    value = samples / (ms / 1e3)
    # the same K strides timed four more times: median of five
    reps = [ms] + [timed(plan, strides, 0, steps, write, False)[0] for _ in range(4)]
    ms_med = float(np.median(reps))
    # per-kernel HIP-event timing over a second timed region (direct launches)
    _, prof = timed(plan, strides, 0, min(steps, 16), write, True)
    kernel_ms = {k: round(v[0] / v[1], 5) for k, v in prof.items() if v[1] > 0}   # the stride's kernels
    kb = kernel_bytes(w, args.precision, write)
    roofs = {}
    for k in ("down", "corr", "mix", "peaks"):
        if k in kernel_ms:
            roofs[k] = roof(kf.get(k, 0.0), kb[k], kernel_ms[k], kernel_peak(args.precision, k))
            roofs[k]["traffic"] = measured_traffic(k, args.workload, args.precision)
    dom = max(("corr", "mix"), key=lambda k: kernel_ms.get(k, 0.0))
    d = roofs[dom]
    if d["bound"] == "hbm":
        top_roof = {"bound": "hbm", "kernel": dom, "achieved": d["hbm_gbs"], "peak": HBM_GBS, "unit": "GB/s",
                    "frac": d["hbm_frac"], "bytes_per_launch": d["bytes"]}
    else:
        top_roof = {"bound": "mfma", "kernel": dom, "achieved": d["mfma_tflops"], "peak": d["mfma_peak"],
                    "unit": "TFLOP/s", "frac": d["mfma_frac"], "flops_per_launch": d["flops"]}
    top_roof["traffic"] = measured_traffic(dom, args.workload, args.precision)
    top_roof["mfma_frac"], top_roof["hbm_frac"] = d["mfma_frac"], d["hbm_frac"]
    # the whole stride against its own bound: all kernels' flops at the MFMA
    # peak of their arithmetic, or all their bytes at the HBM peak
    t_f = sum(kf[k] / (kernel_peak(args.precision, k) * 1e12) for k in ("corr", "mix"))
    t_b = sum(kb.values()) / (HBM_GBS * 1e9)
    stride_roof = {"ms": ms / steps, "mfma_ms": t_f * 1e3, "hbm_ms": t_b * 1e3,
                   "bound": "mfma" if t_f > t_b else "hbm", "frac": max(t_f, t_b) / (ms / steps / 1e3)}

    # peaks-only mode (no series written): the same plan, K strides
    peaks_only = None
    if write and args.peaks_only_leg:
        pms, _ = timed(plan, strides, 0, steps, False, False)
        peaks_only = {"ms_per_step": pms / steps, "value": samples / (pms / 1e3)}
        log(f"peaks only: {pms / steps:.3f} ms per stride")

    xi2 = coinc = None
    if args.xi2 == 1 or (args.xi2 == -1 and args.workload != "largest"):
        m = downstream_measure(plan, w, strides, min(steps, 16))
        gbs = m["bytes"] / (m["ms"] / 1e3) / 1e9
        xi2 = {"ms": m["ms"], "launches": m["launches"], "acf_lengths": m["acf_lengths"], "finite": m["finite"],
               "roofline": {"bound": "hbm", "kernel": "xi2", "achieved": gbs, "peak": HBM_GBS, "unit": "GB/s",
                            "frac": gbs / HBM_GBS, "bytes_per_launch": m["bytes"],
                            "traffic": measured_traffic("xi2", args.workload, args.precision)}}
        tgbs = m["trig_bytes"] / (m["trig_ms"] / 1e3) / 1e9
        coinc = {"overlap_samples": m["overlap"], "window_ms": m["trig_ms"], "coinc_ms": m["coinc_ms"],
                 "banks_with_event": m["events"],
                 "roofline": {"bound": "hbm", "kernel": "window_trigger", "achieved": tgbs, "peak": HBM_GBS,
                              "unit": "GB/s", "frac": tgbs / HBM_GBS, "bytes_per_launch": m["trig_bytes"],
                              "traffic": measured_traffic("window_trigger", args.workload, args.precision)}}
        log(f"xi2: {m['ms']:.4f} ms per launch, {gbs:.0f} GB/s; window triggers {m['trig_ms']:.4f} ms, "
            f"coincidence {m['coinc_ms']:.4f} ms, {m['events']} banks with an event")

    whiten = None
    if args.xi2 == 1 or (args.xi2 == -1 and args.workload != "largest"):
        m = whiten_measure(w, min(steps, 16))
        gbs = m.pop("bytes") / (m["ms_per_push"] / 1e3) / 1e9
        whiten = dict(m, roofline={"bound": "hbm", "kernel": "whitening push", "achieved": gbs, "peak": HBM_GBS,
                                   "unit": "GB/s", "frac": gbs / HBM_GBS, "limited_by": "launch latency",
                                   "traffic": measured_traffic("whitening", args.workload, args.precision)})
        log(f"whitening: {m['ms_per_push']:.4f} ms per push ({m['launches_per_push']} launches), {gbs:.0f} GB/s")

    svd = None
    if args.xi2 == 1 or (args.xi2 == -1 and args.workload != "largest"):
        svd = svd_measure()
        log(f"svd bank construction: {svd['ms']:.2f} ms per slice")

    grad = None
    if args.grad_leg:
        grad = grad_measure(refine_steps=args.refine_steps, tune=bool(args.autotune))
        log(f"gradient: {grad['ms']:.1f} ms per call ({grad['tflops']:.2f} TFLOP/s)")

    base = err = zs = None
    if not args.no_cpu_baseline:
        base, err, zs = parity_and_baseline(plan, w, x, strides, k_par, args.cpu_seconds)
        log(f"oracle sample: {len(zs)} banks, SNR err {err:.3e}")
    flops_per_stride = plan.flops_per_stride
    plan.close()
    del plan
    torch.cuda.synchronize()

    # other forms of the same batched launch (the plain FP32 path; FP16)
    compare = []
    for cp in [c for c in args.compare.split(",") if c and c != args.precision]:
        cplan, cms, _ = run(cp, profile=False)
        cerr = leg_error(cplan, strides, k_par, zs) if zs is not None else None
        compare.append({"precision": cp, "value": samples / (cms / 1e3), "ms_per_step": cms / steps,
                        "snr_err": cerr, "headline_speedup": value / (samples / (cms / 1e3)),
                        "tiling": tiling.get(cp)})
        log(f"{cp}: {steps} strides in {cms:.2f} ms, SNR err {cerr}")
        cplan.close()
        del cplan
    # the unstacked baseline: one plain FP32 plan per bank, launched bank by bank
    loop = None
    if args.loop_leg == 1 or (args.loop_leg == -1 and args.workload == "batched"):
        lms = bank_loop(w, strides, warmup, steps)
        lval = samples / (lms / 1e3)
        loop = {"precision": "fp32", "form": "one plan per bank, launched in a host loop, no graph",
                "value": lval, "ms_per_step": lms / steps, "headline_speedup": value / lval,
                "speedups": {c["precision"]: c["value"] / lval for c in compare}}
        log(f"per-bank FP32 loop: {lms / steps:.3f} ms per stride")

    out = {
        "metric": METRIC, "value": value, "unit": "SNR-samples/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": w.name, "banks": len(w.banks), "templates": w.n_templates, "detectors": ND,
                   "rates_hz": sorted({s.rate for b in w.banks for s in b.slices}, reverse=True),
                   "precision": args.precision, "series_written": write, "graph": bool(args.graph),
                   "stride_s": 1, "flops_per_stride": flops_per_stride, "tiling": tiling.get(args.precision)},
        "roofline": top_roof,
        "stride_roofline": stride_roof,
        "kernel_roofline": roofs,
        "ms_per_step_median5": ms_med / steps,
        "peaks_only": peaks_only,
        "kernel_ms": kernel_ms,
        "xi2": xi2,
        "coincidence": coinc,
        "whitening": whiten,
        "svd_bank": svd,
        "gradient": grad,
        "snr_err": err,
        "compare": compare,
        "baseline_loop": loop,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
