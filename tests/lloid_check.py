"""Helpers shared by the GPU parity tests: run a plan over strides, compare
with the oracle, check triggers."""
from __future__ import annotations

import numpy as np

from oracle import lloid as O


def snr_error(z_gpu: np.ndarray, z_ref: np.ndarray, floor: float = O.SNR_THRESHOLD) -> float:
    """max |z_gpu - z_ref| / max(|z_ref|, floor): relative above the trigger
    threshold, absolute/4 below it."""
    return float((np.abs(z_gpu - z_ref) / np.maximum(np.abs(z_ref), floor)).max())


def run_gpu(plan, x: np.ndarray, first: int, n: int, write_series: bool = True, gaps=None):
    """Push strides 0 .. first+n-1 of x ([n_det, T] float64) and return the
    complex SNR of strides [first, first+n) per bank ([n_det, M, n F]) and
    the peaks per stride per bank."""
    import torch
    F = plan.sample_rate
    xs = torch.from_numpy(np.ascontiguousarray(x.astype(np.float32))).cuda()
    series = plan.new_series() if write_series else None
    peaks = plan.new_peaks()
    z = [[] for _ in range(plan.n_banks)]
    pk = [[] for _ in range(plan.n_banks)]
    for k in range(first + n):
        strain = xs[:, k * F:(k + 1) * F].contiguous()
        mask = gaps[k] if gaps is not None else 0
        plan.push(strain, gap_mask=mask, series=series, peaks=peaks, write_series=write_series)
        if k >= first:
            for b in range(plan.n_banks):
                if write_series:
                    z[b].append(plan.bank_view(series, b).cpu().numpy().astype(np.complex128))
                pk[b].append(plan.peaks_view(peaks, b))
    torch.cuda.synchronize()
    zz = [np.concatenate(v, axis=2) if v else None for v in z]
    return zz, pk


def run_oracle(bank, x: np.ndarray, F: int, first: int, n: int, normalize: bool = True) -> np.ndarray:
    """Oracle complex SNR [n_det, M, n F] for strides [first, first+n)."""
    cfg = O.OracleConfig(F, normalize=normalize)
    out = []
    for d in range(x.shape[0]):
        z, _ = O.lloid_filter(x[d, :(first + n) * F], bank, cfg, n_strides=n, first_stride=first)
        out.append(z)
    return np.stack(out)


def check_peaks(pk, z_ref: np.ndarray, F: int, e_abs: float, threshold: float = 4.0) -> None:
    """Trigger parity per stride: the index is the oracle's unless the oracle
    window holds another sample within 2 e_abs of its maximum, in which case
    it must be one of those; SNR and value agree to the series tolerance."""
    n = z_ref.shape[2] // F
    for k in range(n):
        w = z_ref[:, :, k * F:(k + 1) * F]
        mag = np.abs(w)
        pmax = mag.max(axis=2)
        idx_ref = np.argmax(mag, axis=2)
        p = pk[k]
        near = mag >= (pmax - 2 * e_abs)[..., None]
        ties = near.sum(axis=2) > 1
        exact = ~ties
        assert np.array_equal(p.index[exact], idx_ref[exact]), f"stride {k}: peak index mismatch"
        d_i, m_i = np.nonzero(ties)
        for d, m in zip(d_i, m_i):
            assert near[d, m, p.index[d, m]], f"stride {k}: tied peak index outside the near-max set"
        np.testing.assert_allclose(p.snr, pmax, rtol=0, atol=2 * e_abs + 1e-6 * pmax.max())
        val = w[np.arange(w.shape[0])[:, None], np.arange(w.shape[1])[None, :], p.index]
        np.testing.assert_allclose(p.re, val.real, rtol=0, atol=4 * e_abs + 1e-6)
        np.testing.assert_allclose(p.im, val.imag, rtol=0, atol=4 * e_abs + 1e-6)
        thr_ok = np.abs(pmax - threshold) > 2 * e_abs
        assert np.array_equal(p.above[thr_ok].astype(bool), (pmax >= threshold)[thr_ok])


def _oracle_stride(args):
    bank, x, F, k = args
    from threadpoolctl import threadpool_limits
    cfg = O.OracleConfig(F)
    with threadpool_limits(1):
        return np.stack([O.lloid_filter(x[d], bank, cfg, n_strides=1, first_stride=k)[0] for d in range(x.shape[0])])


def oracle_series(banks, x: np.ndarray, F: int, k: int, workers: int = 16):
    """Oracle complex SNR [n_det, M, F] of stride k for each bank, one bank
    per worker process (one BLAS thread each)."""
    import multiprocessing as mp
    xs = np.ascontiguousarray(x[:, :(k + 1) * F])
    with mp.get_context("spawn").Pool(min(workers, len(banks))) as pool:
        return pool.map(_oracle_stride, [(b, xs, F, k) for b in banks], chunksize=1)
