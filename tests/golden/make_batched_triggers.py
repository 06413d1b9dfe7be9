"""Write the FP64 oracle's triggers of the batched workload (200 uneven
sub-banks, 2 detectors, 4096 Hz) at one steady-state stride, for the GPU
parity test of that workload.  Imports only oracle/ and synth/.

Per bank, detector and template (the plan's peak order) the file holds every
in-stride sample whose |z| lies within TAU = 1e-3 max(p, 4) of the stride
maximum p, largest first (the first entry is the oracle's trigger: the
lowest index attaining p), as (index, re, im); a GPU trigger must be one of
these samples.

    python tests/golden/make_batched_triggers.py [--workers 8]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

STRIDE = 64        # later than the longest filter (64 s): steady state
TAU = 1e-3
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched_triggers_stride64.npz")


def fingerprint(w, x: np.ndarray) -> np.ndarray:
    """Cheap identity of the workload and strain the triggers belong to."""
    F = w.sample_rate
    v = [len(w.banks), w.n_templates, w.n_detectors, F]
    for b in w.banks:
        v += [b.n_templates, len(b.slices)] + [s.delay for s in b.slices] + [s.basis.shape[0] for s in b.slices]
    return np.array([float(np.sum(v)), float(np.sum(np.arange(len(v)) * np.array(v, dtype=np.float64))),
                     float(x[:, STRIDE * F:(STRIDE + 1) * F].sum()),
                     float(sum(b.slices[0].mixing[0, 0] for b in w.banks))])


def _bank(args):
    b, = args
    import synth
    from oracle import lloid as O
    from threadpoolctl import threadpool_limits
    w = synth.cached_workload("c3", synth.config3)
    x = synth.workload_strain(w, STRIDE + 1)
    F = w.sample_rate
    cfg = O.OracleConfig(F)
    out = []
    with threadpool_limits(1):
        for d in range(w.n_detectors):
            z, _ = O.lloid_filter(x[d, :(STRIDE + 1) * F], w.banks[b], cfg, n_strides=1, first_stride=STRIDE)
            mag = np.abs(z)
            p = mag.max(axis=1)
            first = np.argmax(mag, axis=1)
            for i in range(z.shape[0]):
                near = np.nonzero(mag[i] >= p[i] - TAU * max(p[i], 4.0))[0]
                near = near[near != first[i]]
                order = near[np.argsort(-mag[i, near], kind="stable")]
                idx = np.concatenate([[first[i]], order]).astype(np.int32)
                out.append((idx, z[i, idx]))
    return b, out


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    import multiprocessing as mp
    import synth
    w = synth.cached_workload("c3", synth.config3)
    x = synth.workload_strain(w, STRIDE + 1)
    t0 = time.time()
    res = {}
    with mp.get_context("spawn").Pool(args.workers) as pool:
        for b, out in pool.imap_unordered(_bank, [(b,) for b in range(len(w.banks))]):
            res[b] = out
            print(f"bank {b} done ({len(res)} of {len(w.banks)}, {time.time() - t0:.0f} s)", flush=True)
    count, idx, re, im = [], [], [], []
    for b in range(len(w.banks)):
        for ix, zv in res[b]:
            count.append(len(ix))
            idx.append(ix)
            re.append(zv.real)
            im.append(zv.imag)
    np.savez_compressed(OUT, stride=STRIDE, tau=TAU, fingerprint=fingerprint(w, x),
                        count=np.array(count, dtype=np.int32), index=np.concatenate(idx).astype(np.int32),
                        re=np.concatenate(re).astype(np.float32), im=np.concatenate(im).astype(np.float32))
    print(f"wrote {OUT}: {len(count)} triggers, {sum(count)} samples", flush=True)


if __name__ == "__main__":
    main()
