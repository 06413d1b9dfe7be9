"""Seeded synthetic workloads for the LLOID filtering core.

This module produces *inputs only*: whitened Gaussian strain, injected
chirps, and compressed template banks (per-slice basis filters U^s and
mixing matrices W^s).  It holds none of the filtering arithmetic (resampling,
correlation, reconstruction, upsampling, peak finding, normalisation); both
the FP64 oracle and the GPU path consume what it returns.

Bank construction follows the SVD bank recipe of Sec. II.C.1 (time slicing,
per-slice sample rate, SVD with truncation to the leading L^s bases, Eq. for
the decomposition h ~ sum_l v sigma u).  It is offline input preparation,
not part of the per-stride filtering path.

Every random draw comes from ``numpy.random.default_rng([config, purpose,
index])`` with purpose 0 = noise, 1 = bank, 2 = injections, 3 = sub-bank
structure, so every workload is reproducible from its config number.

The paper measures on replayed O3 detector data with the O4 template bank;
neither is available here.  The workloads below stand in for them with
unit-variance whitened Gaussian noise, Newtonian-chirp banks and seeded
uneven sub-banks of the same structure (rates, slice lengths, basis counts).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

PURPOSE_NOISE, PURPOSE_BANK, PURPOSE_INJ, PURPOSE_STRUCT = 0, 1, 2, 3


def rng_for(config: int, purpose: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(config), int(purpose), int(index)])


@dataclass
class Slice:
    """One time slice of one bank (Sec. II.C.1).

    rate   -- sample rate f^s in Hz (top rate divided by a power of two)
    delay  -- t^s * f^s: time before merger of the slice's latest tap, in
              samples at f^s
    basis  -- U^s, shape [L^s, N^s], float64, taps in chronological order
              (column N^s-1 is the tap closest to merger)
    mixing -- W^s = v*sigma, shape [2M, L^s], float64; row 2i is the cosine
              (real) filter of template i, row 2i+1 the sine (imaginary) one
    """
    rate: int
    delay: int
    basis: np.ndarray
    mixing: np.ndarray

    @property
    def n_taps(self) -> int:
        return int(self.basis.shape[1])

    @property
    def n_basis(self) -> int:
        return int(self.basis.shape[0])


@dataclass
class Bank:
    n_templates: int
    slices: List[Slice]
    # Optional: per-slice un-compressed template matrices H^s [2M, N^s]
    # (kept for small chirp banks; used by full-rank and direct pins).
    templates: Optional[List[np.ndarray]] = None
    # Optional: chirp parameters (tc per template) for brute-force pins.
    tc: Optional[np.ndarray] = None
    f0: Optional[float] = None


@dataclass
class Injection:
    bank: int
    template: int
    detector: int
    merger_sample: int
    amplitude: float


@dataclass
class Workload:
    name: str
    config: int
    sample_rate: int
    n_detectors: int
    duration_s: int
    banks: List[Bank]
    injections: List[Injection] = field(default_factory=list)

    @property
    def n_samples(self) -> int:
        return self.sample_rate * self.duration_s

    @property
    def n_templates(self) -> int:
        return sum(b.n_templates for b in self.banks)


# ---------------------------------------------------------------------------
# Newtonian chirp waveforms
# ---------------------------------------------------------------------------

def tukey_envelope(tau: np.ndarray, tc: float, alpha: float = 0.1) -> np.ndarray:
    """Tukey(alpha) window over the template's own duration tau in [0, tc]."""
    u = np.asarray(tau, dtype=np.float64) / tc
    w = np.zeros_like(u)
    inside = (u >= 0.0) & (u <= 1.0)
    w[inside] = 1.0
    lo = inside & (u < alpha / 2)
    w[lo] = 0.5 * (1.0 - np.cos(2.0 * np.pi * u[lo] / alpha))
    hi = inside & (u > 1.0 - alpha / 2)
    w[hi] = 0.5 * (1.0 - np.cos(2.0 * np.pi * (1.0 - u[hi]) / alpha))
    return w


def chirp_pair(tau: np.ndarray, f0: float, tc: float) -> Tuple[np.ndarray, np.ndarray]:
    """Cosine and sine Newtonian chirp at times ``tau`` before merger.

    Frequency f = f0 * (tau/tc)^(-3/8) (equivalently f0 (1 - t/tc)^(-3/8)
    with t the time since the start); phase obtained by integrating 2 pi f.
    Unit envelope times a Tukey(0.1) taper; zero outside [0, tc].
    """
    tau = np.asarray(tau, dtype=np.float64)
    x = np.clip(tau / tc, 0.0, 1.0)
    phase = 2.0 * np.pi * f0 * tc * 1.6 * (1.0 - x ** 0.625)
    env = tukey_envelope(tau, tc)
    return env * np.cos(phase), env * np.sin(phase)


def full_rate_norms(f0: float, tcs: np.ndarray, rate: int) -> np.ndarray:
    """Per template: (||h_cos||, ||h_sin||) over its samples at the full rate."""
    out = np.empty((len(tcs), 2))
    for i, tc in enumerate(tcs):
        n = int(np.ceil(tc * rate)) + 1
        c, s = chirp_pair(np.arange(n) / rate, f0, tc)
        out[i, 0] = np.sqrt(np.dot(c, c))
        out[i, 1] = np.sqrt(np.dot(s, s))
    return out


def full_rate_templates(bank: Bank, rate: int) -> np.ndarray:
    """Unit-norm real templates h_r(tau_j), tau_j = j/rate, shape [2M, n]."""
    assert bank.tc is not None
    n = int(np.ceil(bank.tc.max() * rate)) + 1
    tau = np.arange(n) / rate
    out = np.empty((2 * bank.n_templates, n))
    for i, tc in enumerate(bank.tc):
        c, s = chirp_pair(tau, bank.f0, tc)
        out[2 * i] = c / np.sqrt(np.dot(c, c))
        out[2 * i + 1] = s / np.sqrt(np.dot(s, s))
    return out


def chirp_bank(top_rate: int, n_templates: int, f0: float, tc_range: Tuple[float, float],
               slices: Sequence[Tuple[int, float, int, int]], seed: Sequence[int],
               keep_templates: bool = False) -> Bank:
    """Time-sliced, SVD-compressed chirp bank (Sec. II.C.1).

    slices: (rate_hz, start_s, n_taps, n_basis) per slice; slice s covers
    times before merger [start_s, start_s + n_taps/rate).  The slice matrix is
    H^s[r, m] = sqrt(D_s) * h_r(start_s + (n_taps - 1 - m)/rate) with
    D_s = top_rate/rate and h_r unit-norm at the top rate.  The SVD
    H^s = V Sigma Vt is truncated to the leading n_basis bases:
    U^s = Vt[:L], W^s = (V Sigma)[:, :L].
    """
    g = np.random.default_rng(list(seed))
    tcs = g.uniform(tc_range[0], tc_range[1], size=n_templates)
    norms = full_rate_norms(f0, tcs, top_rate)
    out_slices: List[Slice] = []
    mats: List[np.ndarray] = []
    for rate, start_s, n_taps, n_basis in slices:
        D = top_rate // rate
        assert D * rate == top_rate and (D & (D - 1)) == 0
        delay = int(round(start_s * rate))
        assert abs(delay - start_s * rate) < 1e-9
        tau = (delay + (n_taps - 1 - np.arange(n_taps))) / rate
        H = np.empty((2 * n_templates, n_taps))
        for i, tc in enumerate(tcs):
            c, s = chirp_pair(tau, f0, tc)
            H[2 * i] = np.sqrt(D) * c / norms[i, 0]
            H[2 * i + 1] = np.sqrt(D) * s / norms[i, 1]
        V, S, Vt = np.linalg.svd(H, full_matrices=False)
        L = int(n_basis)
        out_slices.append(Slice(rate=int(rate), delay=delay,
                                basis=np.ascontiguousarray(Vt[:L]),
                                mixing=np.ascontiguousarray(V[:, :L] * S[:L])))
        if keep_templates:
            mats.append(H)
    return Bank(n_templates=n_templates, slices=out_slices,
                templates=mats if keep_templates else None, tc=tcs, f0=f0)


@dataclass
class BurstParams:
    """Per real row and slice: Hann-windowed sinusoid bursts."""
    freq: np.ndarray      # [2M, S] Hz
    phase: np.ndarray     # [2M, S]
    span: List[Tuple[float, float]]   # per slice: burst support in time before merger (s)
    norm: np.ndarray      # [2M] full-rate norm


def burst_waveform(tau: np.ndarray, p: BurstParams, r: int) -> np.ndarray:
    """Row r of a burst bank at times ``tau`` before merger (unnormalised)."""
    out = np.zeros_like(tau, dtype=np.float64)
    for s, (a, b) in enumerate(p.span):
        u = (tau - a) / (b - a)
        inside = (u >= 0) & (u <= 1)
        w = np.where(inside, np.sin(np.pi * np.clip(u, 0, 1)) ** 2, 0.0)
        out += w * np.cos(2 * np.pi * p.freq[r, s] * tau + p.phase[r, s])
    return out


def burst_bank(top_rate: int, n_templates: int, slices: Sequence[Tuple[int, float, int, int]],
               seed: Sequence[int], band: Tuple[float, float] = (0.02, 0.1)) -> Bank:
    """Smooth, band-limited bank for multirate pins.

    Every real template is a sum of Hann-windowed sinusoid bursts, one per
    slice, each lying strictly inside its slice with frequency in
    band * f^s.  Unlike hard-sliced chirps, each slice's piece is then
    band-limited well below the slice's Nyquist rate, so the multirate filter
    must agree with the top-rate direct filter to within the resamplers'
    passband accuracy.  Rows 2i and 2i+1 differ by a quarter cycle.
    Slices are sampled as in chirp_bank (sqrt(D) scaling) and kept at full
    rank; ``templates`` holds H^s and ``tc`` is left None.
    """
    g = np.random.default_rng(list(seed))
    S = len(slices)
    rows = 2 * n_templates
    freq = np.zeros((rows, S))
    phase = np.zeros((rows, S))
    span = []
    for s, (rate, start, n, _) in enumerate(slices):
        dur = n / rate
        span.append((start + 0.1 * dur, start + 0.9 * dur))
        f = g.uniform(band[0] * rate, band[1] * rate, size=n_templates)
        ph = g.uniform(0, 2 * np.pi, size=n_templates)
        freq[0::2, s] = f
        freq[1::2, s] = f
        phase[0::2, s] = ph
        phase[1::2, s] = ph - np.pi / 2
    T = max(st + n / r for r, st, n, _ in slices)
    tau = np.arange(int(np.ceil(T * top_rate)) + 1) / top_rate
    p = BurstParams(freq, phase, span, np.ones(rows))
    p.norm = np.array([np.sqrt(np.sum(burst_waveform(tau, p, r) ** 2)) for r in range(rows)])
    out, mats = [], []
    for rate, start, n_taps, n_basis in slices:
        D = top_rate // rate
        delay = int(round(start * rate))
        tt = (delay + (n_taps - 1 - np.arange(n_taps))) / rate
        H = np.stack([np.sqrt(D) * burst_waveform(tt, p, r) / p.norm[r] for r in range(rows)])
        V, S_, Vt = np.linalg.svd(H, full_matrices=False)
        L = min(int(n_basis), len(S_))
        out.append(Slice(int(rate), delay, np.ascontiguousarray(Vt[:L]),
                         np.ascontiguousarray(V[:, :L] * S_[:L])))
        mats.append(H)
    bank = Bank(n_templates, out, mats)
    bank.burst = p
    return bank


def burst_full_rate(bank: Bank, top_rate: int) -> np.ndarray:
    """Unit-norm top-rate samples h_r(j/F) of a burst bank, [2M, n]."""
    p = bank.burst
    T = max(b for _, b in p.span)
    tau = np.arange(int(np.ceil(T * top_rate)) + 1) / top_rate
    return np.stack([burst_waveform(tau, p, r) / p.norm[r] for r in range(len(p.norm))])


def truncate_bank(bank: Bank, n_basis: Sequence[int]) -> Bank:
    """Same bank keeping only the leading n_basis[s] bases of every slice."""
    sl = [Slice(s.rate, s.delay, np.ascontiguousarray(s.basis[:L]),
                np.ascontiguousarray(s.mixing[:, :L])) for s, L in zip(bank.slices, n_basis)]
    return Bank(bank.n_templates, sl, bank.templates, bank.tc, bank.f0)


# ---------------------------------------------------------------------------
# Random uneven sub-banks (batched workloads)
# ---------------------------------------------------------------------------

def slice_lookahead_s(rates_desc: Sequence[int], r: int, n_down: int = 32, n_up: int = 8) -> float:
    """Seconds of look-ahead a slice at rates_desc[r] needs (sub-bank layout
    rule only): downsampling half-length plus the upsampling half-lengths of
    every stage between its rate and the top rate."""
    if r == 0:
        return 0.0
    return n_down / rates_desc[r] + sum(n_up / rates_desc[j] for j in range(1, r + 1))


def subbank_shape(g: np.random.Generator, top_rate: int, n_rates_range: Tuple[int, int],
                  templates_range: Tuple[int, int], duration_range: Tuple[float, float]):
    """The first draws of a sub-bank: templates M, rate count R, the rates,
    the per-rate lower bounds of the slice boundaries and the duration T."""
    M = int(g.integers(templates_range[0], templates_range[1] + 1))
    R = int(g.integers(n_rates_range[0], n_rates_range[1] + 1))
    rates = [top_rate >> r for r in range(R)]
    tmin = [0.0] + [np.ceil(1.5 * slice_lookahead_s(rates, r) * rates[r]) / rates[r] for r in range(1, R)]
    lo = max(duration_range[0], 2.0 * tmin[R - 1])
    T = float(np.exp(g.uniform(np.log(lo), np.log(max(lo, duration_range[1])))))
    return M, R, rates, tmin, T


def subbank_boundaries(rates: Sequence[int], tmin: Sequence[float], T: float) -> List[float]:
    """Slice boundaries tau_0 = 0 < tau_1 < ... < tau_R = T in seconds, each
    on its rate's sample grid."""
    R = len(rates)
    taus = [0.0]
    for r in range(1, R):
        t = max(tmin[r], T * 4.0 ** (-(R - r)))
        taus.append(np.round(t * rates[r]) / rates[r])
    taus.append(np.round(T * rates[R - 1]) / rates[R - 1])
    return taus


def random_subbank(g: np.random.Generator, top_rate: int, n_rates_range: Tuple[int, int],
                   templates_range: Tuple[int, int], duration_range: Tuple[float, float],
                   basis_range: Tuple[int, int], dtype=np.float64) -> Bank:
    """One uneven sub-bank: random orthonormal bases and decaying mixing rows.

    rates top/2^r, r < R; slice boundaries tau_r = max(tau_r^min, T 4^-(R-r))
    on the 1/f_r grid, with tau_r^min = 1.5 x the slice's look-ahead; T is
    log-uniform; L_r uniform and clipped to min(N_r, 2M).  Bases are the Q of
    a Gaussian QR; W rows are Gaussian x exp(-3 l / L), rows jointly
    normalised over slices.
    """
    M, R, rates, tmin, T = subbank_shape(g, top_rate, n_rates_range, templates_range, duration_range)
    taus = subbank_boundaries(rates, tmin, T)
    slices = []
    rows = []
    for r in range(R):
        N = int(round((taus[r + 1] - taus[r]) * rates[r]))
        assert N >= 1
        L = int(g.integers(basis_range[0], basis_range[1] + 1))
        L = min(L, N, 2 * M)
        Q, _ = np.linalg.qr(g.standard_normal((N, L)))
        sig = np.exp(-3.0 * np.arange(L) / L)
        W = g.standard_normal((2 * M, L)) * sig
        rows.append(W)
        slices.append(Slice(rate=rates[r], delay=int(round(taus[r] * rates[r])),
                            basis=np.ascontiguousarray(Q.T.astype(dtype)), mixing=W))
    nrm = np.sqrt(sum((W * W).sum(axis=1) for W in rows))
    for s in slices:
        s.mixing = np.ascontiguousarray((s.mixing / nrm[:, None]).astype(dtype))
    return Bank(n_templates=M, slices=slices)


# ---------------------------------------------------------------------------
# Autocorrelation inputs of the xi^2 statistic (seeded stand-ins)
# ---------------------------------------------------------------------------

ACF_SHORT, ACF_LONG = 351, 701   # full autocorrelation lengths for high- and low-mass templates


def acf_length(bank: Bank) -> int:
    """ACF_SHORT for banks whose templates last at most 8 s, ACF_LONG beyond."""
    dur = max((s.delay + s.basis.shape[1]) / s.rate for s in bank.slices)
    return ACF_LONG if dur > 8.0 else ACF_SHORT


def synthetic_acf(config: int, index: int, n_templates: int, length: int) -> np.ndarray:
    """Seeded chirp-like autocorrelations, complex [M, length], t = -(length-1)/2
    .. (length-1)/2: R(t) = exp(-(t/w)^2/2) exp(-i (a t + b t |t|)) with
    per-template width w, frequency a and sweep b.  R(0) = 1, |R| <= 1 and
    R(-t) = conj R(t), as for a template's own autocorrelation."""
    g = rng_for(config, PURPOSE_STRUCT, 1000 + index)
    t = np.arange(length) - (length - 1) // 2
    w = g.uniform(5.0, 60.0, n_templates)[:, None]
    a = g.uniform(0.05, 1.5, n_templates)[:, None]
    b = g.uniform(-2e-3, 2e-3, n_templates)[:, None]
    return np.exp(-0.5 * (t / w) ** 2) * np.exp(-1j * (a * t + b * t * np.abs(t)))


# ---------------------------------------------------------------------------
# Strain and injections
# ---------------------------------------------------------------------------

def gaussian_strain(config: int, n_detectors: int, n_samples: int) -> np.ndarray:
    """Unit-variance whitened Gaussian noise, float64 [n_det, n_samples]."""
    return np.stack([rng_for(config, PURPOSE_NOISE, d).standard_normal(n_samples)
                     for d in range(n_detectors)])


def inject(strain: np.ndarray, top_rate: int, bank: Bank, inj: Injection) -> None:
    """Add A * h_cos(tau_j) of a chirp template at sample merger - j, in place."""
    tc = bank.tc[inj.template]
    n = int(np.ceil(tc * top_rate)) + 1
    c, _ = chirp_pair(np.arange(n) / top_rate, bank.f0, tc)
    c = c / np.sqrt(np.dot(c, c))
    t = inj.merger_sample - np.arange(n)
    ok = (t >= 0) & (t < strain.shape[1])
    strain[inj.detector, t[ok]] += inj.amplitude * c[ok]


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

C1_SLICES = [(2048, 0.0, 1024, 16), (512, 0.5, 1792, 16)]
C2_SLICES = [(4096, 0.0, 1024, 40), (2048, 0.25, 1536, 60), (1024, 1.0, 3072, 80),
             (512, 4.0, 6144, 100), (256, 16.0, 12288, 120)]
C4_BASIS = [20, 30, 40, 50, 60]


def config1(keep_templates: bool = True) -> Workload:
    """Plain LLOID: 1 detector, 32 s at 2048 Hz, 64 chirps (f0=30 Hz,
    tc in [2,4] s), 2 rates, L=16 per rate, one injection with amplitude 12."""
    bank = chirp_bank(2048, 64, 30.0, (2.0, 4.0), C1_SLICES, seed=[1, PURPOSE_BANK, 0],
                      keep_templates=keep_templates)
    g = rng_for(1, PURPOSE_INJ)
    j = int(g.integers(64))
    t0 = int(g.integers(8 * 2048, 28 * 2048))
    return Workload("plain-64x2rates-2048Hz-32s", 1, 2048, 1, 32, [bank],
                    [Injection(0, j, 0, t0, 12.0)])


def config2(duration_s: int = 4096, keep_templates: bool = False, n_basis=None) -> Workload:
    """Single realistic bank: 1 detector, 4096 s at 4096 Hz, 1024 chirps
    (f0=15 Hz, tc in [8,64] s), 5 rates, L = 40/60/80/100/120, 20 injections
    with amplitude in [8, 20]."""
    bank = chirp_bank(4096, 1024, 15.0, (8.0, 64.0), C2_SLICES, seed=[2, PURPOSE_BANK, 0],
                      keep_templates=keep_templates)
    if n_basis is not None:
        bank = truncate_bank(bank, n_basis)
    g = rng_for(2, PURPOSE_INJ)
    injs = []
    for _ in range(20):
        j = int(g.integers(1024))
        t0 = int(g.integers(64 * 4096, 4096 * 4096))
        a = float(g.uniform(8.0, 20.0))
        if t0 < duration_s * 4096:
            injs.append(Injection(0, j, 0, t0, a))
    return Workload("single-bank-1024x5rates-4096Hz", 2, 4096, 1, duration_s, [bank], injs)


def config4(duration_s: int = 64) -> Workload:
    """Gradient workload: the realistic bank truncated to 50 % of its basis
    counts (20/30/40/50/60), 64 s at 4096 Hz, 1 detector."""
    w = config2(duration_s=duration_s, keep_templates=True, n_basis=C4_BASIS)
    w.name = "gradient-1024x5rates-halfbasis-4096Hz"
    w.config = 4
    return w


def batched_banks(config: int, n_banks: int, n_rates_range, duration_range,
                  dtype=np.float64, progress=None) -> List[Bank]:
    """Sub-banks drawn one after another from one generator (the batched
    workload's banks)."""
    g = rng_for(config, PURPOSE_STRUCT)
    banks = []
    for i in range(n_banks):
        banks.append(random_subbank(g, 4096, n_rates_range, (200, 1000), duration_range, (20, 150), dtype))
        if progress is not None and (i + 1) % 100 == 0:
            progress(f"generated {i + 1} of {n_banks} banks")
    return banks


# the largest workload draws every sub-bank from its own generator, so that a
# test can build any subset of its banks without generating the rest
C5_RATES, C5_DURATION = (3, 6), (0.5, 128.0)


def _c5_rng(i: int) -> np.random.Generator:
    return rng_for(5, PURPOSE_STRUCT, i + 1)


def config5_shapes(n_banks: int = 800) -> List[Tuple[int, int, float, int]]:
    """(templates, rates, duration in s, longest slice in taps) of every
    sub-bank of the largest workload, from the first draws of its generator
    only."""
    out = []
    for i in range(n_banks):
        M, R, rates, tmin, T = subbank_shape(_c5_rng(i), 4096, C5_RATES, (200, 1000), C5_DURATION)
        taus = subbank_boundaries(rates, tmin, T)
        nmax = max(int(round((taus[r + 1] - taus[r]) * rates[r])) for r in range(R))
        out.append((M, R, T, nmax))
    return out


def config5_banks(indices: Sequence[int], dtype=np.float64, progress=None) -> List[Bank]:
    """The largest workload's sub-banks with the given indices."""
    banks = []
    for n, i in enumerate(indices):
        banks.append(random_subbank(_c5_rng(int(i)), 4096, C5_RATES, (200, 1000), C5_DURATION, (20, 150), dtype))
        if progress is not None and (n + 1) % 100 == 0:
            progress(f"generated {n + 1} of {len(indices)} banks")
    return banks


def config3(n_banks: int = 200, duration_s: int = 256) -> Workload:
    """Batched uneven sub-banks: 2 detectors, 256 s at 4096 Hz, 200 banks of
    200-1000 templates, 3-7 rates, L in [20,150], filters 0.5-64 s."""
    return Workload("batched-200banks-2det-4096Hz", 3, 4096, 2, duration_s,
                    batched_banks(3, n_banks, (3, 7), (0.5, 64.0)))


def config5(n_banks: int = 800, duration_s: int = 1024, dtype=np.float64, progress=None) -> Workload:
    """Largest single-GPU share: 2 detectors, 1024 s at 4096 Hz, 800 uneven
    sub-banks (up to 6 rates, lowest 128 Hz, filters up to 128 s)."""
    return Workload("batched-800banks-2det-4096Hz", 5, 4096, 2, duration_s,
                    config5_banks(range(n_banks), dtype, progress))


CACHE_VERSION = 1


def _cache_dir() -> str:
    import os
    import tempfile
    d = os.environ.get("LLOID_SYNTH_CACHE", os.path.join(tempfile.gettempdir(), "lloid_synth_cache"))
    os.makedirs(d, exist_ok=True)
    return d


def cached_workload(name: str, builder) -> Workload:
    """Build a workload once per machine: banks are stored as .npz (no
    pickles) under $LLOID_SYNTH_CACHE (default: the temp directory)."""
    import json
    import os
    path = os.path.join(_cache_dir(), f"{name}-v{CACHE_VERSION}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"]))
            banks = []
            for b, bm in enumerate(meta["banks"]):
                sl = [Slice(r, d, z[f"U_{b}_{i}"], z[f"W_{b}_{i}"]) for i, (r, d) in enumerate(bm["slices"])]
                tc = z[f"tc_{b}"] if f"tc_{b}" in z else None
                banks.append(Bank(bm["M"], sl, None, tc, bm.get("f0")))
            injs = [Injection(*i) for i in meta["injections"]]
            return Workload(meta["name"], meta["config"], meta["rate"], meta["n_det"], meta["duration"], banks, injs)
    w = builder()
    arrays = {}
    meta = {"name": w.name, "config": w.config, "rate": w.sample_rate, "n_det": w.n_detectors,
            "duration": w.duration_s, "banks": [],
            "injections": [[i.bank, i.template, i.detector, i.merger_sample, i.amplitude] for i in w.injections]}
    for b, bank in enumerate(w.banks):
        meta["banks"].append({"M": bank.n_templates, "f0": bank.f0,
                              "slices": [[s.rate, s.delay] for s in bank.slices]})
        for i, s in enumerate(bank.slices):
            arrays[f"U_{b}_{i}"] = s.basis
            arrays[f"W_{b}_{i}"] = s.mixing
        if bank.tc is not None:
            arrays[f"tc_{b}"] = bank.tc
    tmp = path + f".{os.getpid()}.tmp.npz"
    np.savez(tmp, meta=json.dumps(meta), **arrays)
    os.replace(tmp, path)
    return w


def workload_strain(w: Workload, duration_s: Optional[int] = None) -> np.ndarray:
    """Noise plus the workload's injections, float64 [n_det, rate*duration]."""
    n = w.sample_rate * (duration_s if duration_s is not None else w.duration_s)
    x = gaussian_strain(w.config, w.n_detectors, n)
    for inj in w.injections:
        inject(x, w.sample_rate, w.banks[inj.bank], inj)
    return x
