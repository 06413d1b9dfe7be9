"""Plain FP64 CPU oracle of the LLOID multirate matched filter.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module;
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the GPU library.  Every step follows the paper
(Sec. II.C, "The LLOID filtering algorithm") in its own order and notation,
in float64, with NumPy matmuls and strided window views as the only library
primitives:

  downsample  d^s  -- Eq. (sinc) kernel, Sec. II.C.2 "Downsampling"
  correlate   y^s_l -- basis cross-correlation, Sec. II.C.2 "Filtering and
                       reconstruction", shifted per the pre-synchronisation
                       equation of Sec. II.C.3
  reconstruct y'^s_i -- mixing with sigma^s_l nu^s_il (same paragraph)
  upsample-and-add  -- Eq. (upsample) polyphase form, Sec. II.C.2
                       "Upsampling SNR segments" / "Combining SNR segments",
                       recursion of the pre-synchronisation equation
  triggers          -- Sec. II.D.1: max |complex SNR| per template per window
  xi^2              -- Sec. II.D.2: signal-consistency statistic at a trigger
  coincidence       -- Sec. II.D.3-4: overlapping trigger windows, coincident
                       events across detectors, one event per sub-bank
  whitening         -- Sec. II.B.2: PSD estimation and whitening with
                       frequency-domain downsampling
  FP8 basis values  -- the e4m3 rounding of the FP8 form (extension), for
                       quantisation-aware refinement

Readings of points the paper leaves open are stated where they are used:

* R1 downsampler gain: Eq. (sinc) fixes g[c]=1 but no normalisation.  We use
  g_hat = sqrt(D) g / sum(g): unit DC gain times sqrt(D), which pairs with
  slice templates sampled at f^s and scaled by sqrt(D), so a band-limited
  slice gives the same correlation as at the top rate.
* R2 the downsampler goes from the top rate straight to f^s with one kernel
  of factor D = F/f^s (not a cascade of halvings).
* R3 one upsampling stage per pair of consecutive distinct slice rates,
  factor p = their ratio (the top rate is always the last level).
* R4 Eq. (upsample)'s special case y[i] = x[i/f] holds for the zero-phase
  indexing y[i] = sum_k x[floor(i/f) + N_up - k] z_{i mod f}[k]; the causal
  sum as printed delays by N_up input samples.  We take the zero-phase form;
  the N_up look-ahead it needs is exactly what pre-synchronisation absorbs.
* R5 polyphase taps k f + j beyond the kernel's last index 2c are zero.
* R6 N_up counts input (lower-rate) samples: 2 f N_up + 1 taps at the
  output rate, 2 N_up + 1 taps per phase.
* R7 delays in the pre-synchronisation equation are converted to samples at
  f^s; the integer look-ahead of each level follows from the index ranges.
* R8 the correlation output index is the coalescence time: the latest tap
  (n = N^s - 1) meets data t^s before it, so a signal merging at t peaks at t.
* R9 rows 2i / 2i+1 are the cosine (real) and sine (imaginary) filters of
  template i; z_i = rho_2i + i rho_2i+1.
* R10 discrete SNR is sum h d with unit-norm real filters and unit-variance
  strain, so E|z|^2 = 2 in noise (the xi^2 denominator 2 - 2|R|^2 of
  Sec. II.D.2 has the same normalisation).
* R13 the trigger window is the stride; the max is reported for every
  template, with a separate flag for |z| >= 4.
* R14 argmax ties resolve to the lowest index.
* R15 history before the first sample and gap strides are zeros.
* R20 the template autocorrelation R(t) of Sec. II.D.2 (normalised to
  R(0) = 1) is sum_j h[j] conj h[j - t] / sum_j |h[j]|^2 for the complex
  filter h = h_cos + i h_sin in tau order.  With z(t) = sum_j h[j] x[t - j]
  (brute_force's convention) and white unit-variance strain this is
  E[z(t) conj z(0)] / E|z(0)|^2, the choice that makes the xi^2 denominator
  2 - 2|R|^2 the noise expectation of the numerator.
* R21 the xi^2 integrals are sums over top-rate samples t = -delta..delta
  (dt cancels), delta = (A - 1) / 2 for an autocorrelation of odd length A;
  samples outside the available SNR are left out of both sums.
* R22 xi^2 is evaluated at every per-stride peak (R13), with z(0) the SNR
  at the peak index; the threshold flag is left to the caller.
* R23 trigger-finding windows extend into the past: window k covers
  top-rate samples [kF - O, (k+1)F) with O the overlap (light travel time
  plus the coincidence buffer, in samples); the first window is [0, F).
  Indices are reported relative to kF (negative inside the overlap).
* R24 coincidence is per template (the same template in every detector):
  for every detector a whose trigger reaches the threshold, the candidate
  event holds a and every other detector d whose trigger reaches the
  threshold within w[a][d] samples of a's; it is an event if it holds at
  least two detectors; network SNR = sqrt of the sum of the held SNR^2.
  The template's event is its candidate with the largest network SNR
  (lowest anchor detector on ties).
* R25 clustering keeps, per sub-bank and window, the event with the largest
  network SNR (lowest template on ties).  Network SNR^2 is summed in
  detector order in float32, the precision the GPU decides in.
* R26 whitening blocks: N input samples (a power of two), zero padding Z on
  each side, hop H = N/2 - Z; the segment of the last 2H inputs times the
  periodic Hann window sin^2(pi m / 2H), which sums to one at hop H.
  Frequency-domain downsampling by D keeps the first N/(2D) + 1 bins and
  inverts with an N/D-point transform (NumPy's irfft: the imaginary parts
  of the DC and new Nyquist bins are dropped).
* R27 instantaneous PSD per bin: |X_k|^2 / sum(hann^2) (the variance per
  sample for white noise).  The running estimate takes the median of the
  most recent c estimates, c = the largest odd count <= min(blocks seen,
  n_med), divides it by beta_c = exp(E[log median of c unit exponentials]
  + gamma) (median to geometric mean of chi^2_2 bins), and updates the log
  geometric mean by a running average over min(blocks seen, n_avg) blocks;
  PSD = geometric mean x e^gamma.  The current block's estimate is
  included before it is whitened.
* R28 whitened block: Y_k = X_k / sqrt(D PSD_k) (unit variance for white
  noise), inverse transform, times a Tukey window that is one over the
  segment and a raised cosine over each Z/D-sample pad, overlap-added;
  each push outputs the first H/D samples of the accumulator (input times
  [iH - 2H - Z, iH - H - Z) for push i = 1, 2, ...: latency N/2).  A gap
  push adds no block and updates no PSD; the accumulator still drains.
* normalisation: each real row is scaled so that sum_s sum_l W^s[r,l]^2 = 1
  (the reconstructed template has unit norm), computed in float64.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

N_DOWN = 32       # downsampler half-length at the target rate (Sec. II.C.2)
N_UP = 8          # upsampler half-length in input samples (Sec. II.C.2)
SNR_THRESHOLD = 4.0   # trigger threshold (Sec. II.D.1)


@dataclass
class OracleConfig:
    sample_rate: int
    n_down: int = N_DOWN
    n_up: int = N_UP
    normalize: bool = True
    snr_threshold: float = SNR_THRESHOLD


# ---------------------------------------------------------------------------
# Resampling kernels (Eq. (sinc), Sec. II.C.2)
# ---------------------------------------------------------------------------

def sinc_windowed_sinc(f: int, c: int) -> np.ndarray:
    """g[k] = sinc((k-c)/f) * sinc((k-c)/c), k = 0..2c, g[c] = 1 (Eq. (sinc)).

    numpy's sinc(x) = sin(pi x)/(pi x) with sinc(0) = 1, which is the form of
    both factors of the equation."""
    u = np.arange(2 * c + 1, dtype=np.float64) - c
    return np.sinc(u / f) * np.sinc(u / c)


def downsample_kernel(D: int, n_down: int = N_DOWN) -> Tuple[np.ndarray, int]:
    """Normalised decimation kernel g_hat = sqrt(D) g / sum g, c = D N_down
    (reading R1)."""
    c = D * n_down
    g = sinc_windowed_sinc(D, c)
    return np.sqrt(D) * g / g.sum(), c


def upsample_kernel(p: int, n_up: int = N_UP) -> Tuple[np.ndarray, int]:
    """Interpolation kernel: Eq. (sinc) with factor p and c = p N_up,
    unnormalised (g[c] = 1), 2 p N_up + 1 taps (reading R6)."""
    c = p * n_up
    return sinc_windowed_sinc(p, c), c


def polyphase_subkernels(p: int, n_up: int = N_UP) -> np.ndarray:
    """z_j[k] = g[k p + j], j < p, k = 0..2 N_up; zero past 2c (reading R5)."""
    g, c = upsample_kernel(p, n_up)
    z = np.zeros((p, 2 * n_up + 1))
    for j in range(p):
        for k in range(2 * n_up + 1):
            if k * p + j <= 2 * c:
                z[j, k] = g[k * p + j]
    return z


# ---------------------------------------------------------------------------
# Index helpers
# ---------------------------------------------------------------------------

def take(x: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """x[..., lo:hi] with zeros outside x's support (reading R15)."""
    n = x.shape[-1]
    out = np.zeros(x.shape[:-1] + (hi - lo,), dtype=np.float64)
    a, b = max(lo, 0), min(hi, n)
    if b > a:
        out[..., a - lo:b - lo] = x[..., a:b]
    return out


def rate_chain(bank, top_rate: int) -> List[int]:
    """Distinct slice rates in decreasing order, starting at the top rate
    (reading R3)."""
    rates = sorted({int(s.rate) for s in bank.slices} | {int(top_rate)}, reverse=True)
    for r in rates:
        if top_rate % r or (top_rate // r) & (top_rate // r - 1):
            raise ValueError(f"rate {r} is not the top rate over a power of two")
    return rates


def level_ranges(chain: Sequence[int], t_lo: int, t_hi: int, n_up: int = N_UP) -> List[Tuple[int, int]]:
    """Index range [lo_j, hi_j) of each level's stream needed for top-rate
    outputs [t_lo, t_hi): the zero-phase polyphase sum at level j-1 reads
    level j from floor(i/p) - N_up to floor(i/p) + N_up."""
    out = [(t_lo, t_hi)]
    for j in range(1, len(chain)):
        p = chain[j - 1] // chain[j]
        lo, hi = out[-1]
        out.append((lo // p - n_up, (hi - 1) // p + n_up + 1))
    return out


def lookahead(chain: Sequence[int], n_up: int = N_UP) -> List[int]:
    """Samples at level j beyond the end of the current stride that level j
    must supply: the cumulative upsampling half-lengths of the
    pre-synchronisation equation (Sec. II.C.3) in level-j samples."""
    F = chain[0]
    rng = level_ranges(chain, 0, F, n_up)
    return [hi - r for (lo, hi), r in zip(rng, chain)]


def latency_violations(bank, top_rate: int, n_down: int = N_DOWN, n_up: int = N_UP) -> List[int]:
    """Slices whose delay is shorter than the downsampling plus cumulative
    upsampling look-ahead (Sec. II.C.2 "Combining SNR segments": no extra
    latency as long as the delays exceed the filter lengths).  Such a slice
    would need strain from the future of the current stride."""
    chain = rate_chain(bank, top_rate)
    la = lookahead(chain, n_up)
    bad = []
    for i, s in enumerate(bank.slices):
        j = chain.index(int(s.rate))
        need = la[j] + (n_down if s.rate != top_rate else 0)
        if s.delay < need:
            bad.append(i)
    return bad


# ---------------------------------------------------------------------------
# The steps
# ---------------------------------------------------------------------------

def normalized_mixing(bank) -> List[np.ndarray]:
    """W~^s = W^s / n_r, n_r^2 = sum_s sum_l W^s[r,l]^2 in float64."""
    n2 = sum((np.asarray(s.mixing, np.float64) ** 2).sum(axis=1) for s in bank.slices)
    n = np.sqrt(n2)
    n[n == 0] = 1.0
    return [np.asarray(s.mixing, np.float64) / n[:, None] for s in bank.slices]


def downsample(x: np.ndarray, D: int, m_lo: int, m_hi: int, n_down: int = N_DOWN) -> np.ndarray:
    """d_D[m] = sum_{k=0}^{2c} g_hat[k] x[D m + k - c], m in [m_lo, m_hi)
    (Eq. (sinc) kernel, zero-phase; readings R1, R2)."""
    if D == 1:
        return take(x, m_lo, m_hi)
    g, c = downsample_kernel(D, n_down)
    seg = take(x, D * m_lo - c, D * (m_hi - 1) + c + 1)
    win = sliding_window_view(seg, 2 * c + 1)[::D]      # win[i, k] = x[D(m_lo+i) - c + k]
    return win @ g


def correlate(U: np.ndarray, d: np.ndarray, d_lo: int, delay: int, q_lo: int, q_hi: int) -> np.ndarray:
    """y_l[q] = sum_{n<N} u_l[n] d[q - delay - (N-1) + n], q in [q_lo, q_hi).

    The basis correlation of Sec. II.C.2 with the slice delay of the
    pre-synchronisation equation; index q is the coalescence time (R8).
    ``d`` holds the downsampled stream starting at index d_lo."""
    L, N = U.shape
    a = q_lo - delay - (N - 1) - d_lo
    seg = d[a:a + (q_hi - q_lo) + N - 1]
    assert a >= 0 and seg.shape[0] == (q_hi - q_lo) + N - 1
    H = sliding_window_view(seg, N)                     # H[i, n] = d[q_lo + i - delay - N + 1 + n]
    return U @ H.T


def upsample(a: np.ndarray, a_lo: int, p: int, i_lo: int, i_hi: int, n_up: int = N_UP) -> np.ndarray:
    """(H_up a)[i] = sum_{k=0}^{2 N_up} a[floor(i/p) + N_up - k] z_{i mod p}[k]
    for i in [i_lo, i_hi) (Eq. (upsample), zero-phase reading R4).
    ``a`` is [rows, n] holding indices a_lo .. a_lo + n - 1."""
    z = polyphase_subkernels(p, n_up)
    i = np.arange(i_lo, i_hi)
    q, ph = i // p, i % p
    out = np.zeros((a.shape[0], i_hi - i_lo))
    for k in range(2 * n_up + 1):
        src = q + n_up - k - a_lo
        assert src.min() >= 0 and src.max() < a.shape[1]
        out += a[:, src] * z[ph, k][None, :]
    # the equation's first case: phase-0 outputs are the input samples
    zero = ph == 0
    out[:, zero] = a[:, q[zero] - a_lo]
    return out


def snr_series(x: np.ndarray, bank, cfg: OracleConfig, t_lo: int, t_hi: int,
               mixing: Optional[List[np.ndarray]] = None) -> np.ndarray:
    """Real SNR streams rho[r, t] for top-rate times t in [t_lo, t_hi).

    x is one detector's whitened strain at the top rate (zero outside its
    support).  Lowest rate first: A_J = sum of z^s at R_J; then
    A_j = H_up(A_{j+1}) + sum_{f^s = R_j} z^s, z^s = W~^s y^s, up to the top
    rate (recursion of the pre-synchronisation equation, Sec. II.C.3)."""
    F = cfg.sample_rate
    chain = rate_chain(bank, F)
    ranges = level_ranges(chain, t_lo, t_hi, cfg.n_up)
    if mixing is None:
        mixing = normalized_mixing(bank) if cfg.normalize else [np.asarray(s.mixing, np.float64) for s in bank.slices]
    rows = 2 * bank.n_templates
    # one downsampled stream per distinct rate, over the union of needed indices
    need: Dict[int, Tuple[int, int]] = {}
    for s in bank.slices:
        j = chain.index(int(s.rate))
        lo, hi = ranges[j]
        a, b = lo - s.delay - (s.n_taps - 1), hi - s.delay
        if s.rate in need:
            a, b = min(a, need[s.rate][0]), max(b, need[s.rate][1])
        need[s.rate] = (a, b)
    streams = {r: (a, downsample(x, F // r, a, b, cfg.n_down)) for r, (a, b) in need.items()}
    A = None
    for j in range(len(chain) - 1, -1, -1):
        lo, hi = ranges[j]
        acc = np.zeros((rows, hi - lo))
        if A is not None:
            acc += upsample(A, ranges[j + 1][0], chain[j] // chain[j + 1], lo, hi, cfg.n_up)
        for s, W in zip(bank.slices, mixing):
            if s.rate != chain[j]:
                continue
            d_lo, d = streams[s.rate]
            y = correlate(np.asarray(s.basis, np.float64), d, d_lo, s.delay, lo, hi)
            acc += W @ y
        A = acc
    return A


def complex_snr(rho: np.ndarray) -> np.ndarray:
    """z_i = rho_{2i} + i rho_{2i+1} (reading R9)."""
    return rho[0::2] + 1j * rho[1::2]


@dataclass
class Peaks:
    snr: np.ndarray      # max |z| per template
    index: np.ndarray    # lowest index attaining it, within the window
    value: np.ndarray    # complex z at that index
    above: np.ndarray    # snr >= threshold


def window_peaks(z: np.ndarray, threshold: float = SNR_THRESHOLD) -> Peaks:
    """Trigger per template over one window (Sec. II.D.1): maximum modulus of
    the complex SNR, its first index, the value there, and the >= rho flag."""
    p2 = z.real ** 2 + z.imag ** 2
    idx = np.argmax(p2, axis=1)
    val = z[np.arange(z.shape[0]), idx]
    snr = np.abs(val)
    return Peaks(snr, idx, val, snr >= threshold)


def lloid_filter(x: np.ndarray, bank, cfg: OracleConfig, n_strides: Optional[int] = None,
                 first_stride: int = 0) -> Tuple[np.ndarray, List[Peaks]]:
    """Batch form: complex SNR for strides [first, first + n) of 1 s each and
    their per-stride triggers.  x is [n_samples] (one detector)."""
    F = cfg.sample_rate
    if n_strides is None:
        n_strides = x.shape[-1] // F - first_stride
    zs, pk = [], []
    for k in range(first_stride, first_stride + n_strides):
        z = complex_snr(snr_series(x, bank, cfg, k * F, (k + 1) * F))
        zs.append(z)
        pk.append(window_peaks(z, cfg.snr_threshold))
    return np.concatenate(zs, axis=1) if zs else np.zeros((bank.n_templates, 0), complex), pk


class LloidStream:
    """Streaming form: push strides in order; each push returns the complex
    SNR for the pushed interval, computed from the strain received so far only
    (the future is unknown and taken as zero).  Equals the batch form exactly
    when no slice violates the latency condition."""

    def __init__(self, bank, cfg: OracleConfig, n_samples_hint: int = 0):
        self.bank, self.cfg = bank, cfg
        self.x = np.zeros(0)
        self.mixing = normalized_mixing(bank) if cfg.normalize else None

    def push(self, chunk: np.ndarray, gap: bool = False) -> np.ndarray:
        chunk = np.zeros(len(chunk)) if gap else np.asarray(chunk, np.float64)
        t0 = self.x.shape[0]
        self.x = np.concatenate([self.x, chunk])
        rho = snr_series(self.x, self.bank, self.cfg, t0, self.x.shape[0], self.mixing)
        return complex_snr(rho)

    def state(self) -> np.ndarray:
        return self.x.copy()

    def load(self, state: np.ndarray) -> None:
        self.x = state.copy()


# ---------------------------------------------------------------------------
# Direct matched filter (Eq. of Sec. II.C, discrete form) for pins
# ---------------------------------------------------------------------------

def brute_force(x: np.ndarray, templates: np.ndarray, t_lo: int, t_hi: int) -> np.ndarray:
    """rho_r[t] = sum_j h_r(tau_j) x[t - j] at the top rate, tau_j = j/F
    (the time-domain matched filter with whitened data and templates,
    discrete, readings R8 and R10).  templates: [2M, n]."""
    n = templates.shape[1]
    seg = take(x, t_lo - n + 1, t_hi)
    H = sliding_window_view(seg, n)          # H[i, m] = x[t_lo + i - n + 1 + m]
    return templates[:, ::-1] @ H.T          # m = n-1-j


def concatenated_filters(bank, top_rate: int, mixing: Optional[List[np.ndarray]] = None) -> np.ndarray:
    """For a bank whose slices are all at the top rate: the full-rate filters
    h_r(tau_j) obtained by placing W~^s U^s at delays t^s (reversed to
    tau order).  Used to pin correlation + mixing + slicing + delays."""
    if mixing is None:
        mixing = [np.asarray(s.mixing, np.float64) for s in bank.slices]
    n = max(s.delay + s.n_taps for s in bank.slices)
    out = np.zeros((2 * bank.n_templates, n))
    for s, W in zip(bank.slices, mixing):
        assert s.rate == top_rate
        R = W @ np.asarray(s.basis, np.float64)        # [2M, N], chronological taps
        out[:, s.delay:s.delay + s.n_taps] += R[:, ::-1]   # tau index j = delay + N-1-m
    return out


# ---------------------------------------------------------------------------
# Gradient of the SNR-reconstruction loss (bank refinement; not in the paper)
# ---------------------------------------------------------------------------

def upsample_adjoint(g: np.ndarray, g_lo: int, p: int, a_lo: int, a_hi: int, n_up: int = N_UP) -> np.ndarray:
    """Transpose of `upsample`: the forward adds a[floor(i/p) + N_up - k] z_{i mod p}[k]
    to output i (phase-0 outputs copy a[i/p]); the transpose adds g[i] times the
    same weight to position floor(i/p) + N_up - k.  g covers level indices
    g_lo .. g_lo + n - 1; returns the lower-rate array over [a_lo, a_hi)."""
    z = polyphase_subkernels(p, n_up)
    i = np.arange(g_lo, g_lo + g.shape[1])
    q, ph = i // p, i % p
    out = np.zeros((g.shape[0], a_hi - a_lo))
    for k in range(2 * n_up + 1):
        w = z[ph, k].copy()
        w[ph == 0] = 1.0 if k == n_up else 0.0
        dst = q + n_up - k - a_lo
        assert dst.min() >= 0 and dst.max() < out.shape[1]
        np.add.at(out.T, dst, (g * w[None, :]).T)
    return out


def _upsample_to_top(a: np.ndarray, chain, ranges, j: int, n_up: int) -> np.ndarray:
    """Apply the upsampling stages from level j to the top level."""
    for i in range(j, 0, -1):
        a = upsample(a, ranges[i][0], chain[i - 1] // chain[i], ranges[i - 1][0], ranges[i - 1][1], n_up)
    return a


def _adjoint_to_level(g: np.ndarray, chain, ranges, j: int, n_up: int) -> np.ndarray:
    """Apply the transposed upsampling stages from the top level down to level j."""
    for i in range(1, j + 1):
        g = upsample_adjoint(g, ranges[i - 1][0], chain[i - 1] // chain[i], ranges[i][0], ranges[i][1], n_up)
    return g


def loss_and_grad(x: np.ndarray, bank, target: np.ndarray, cfg: OracleConfig, t_lo: int, t_hi: int):
    """L = sum_{r, t in [t_lo, t_hi)} (rho[r,t] - target[r,t])^2, rho the LLOID
    output of the bank's own W and U (no row normalisation), and its gradient:

      dL/dW^s[r,l] = 2 sum_t R[r,t] (Up_s y^s_l)[t]
      dL/dU^s[l,n] = 2 sum_q (Up_s^T W^s^T R)[l,q] d^s[q - delay - (N-1) + n]

    with R = rho - target and Up_s the upsampling stages from the slice's
    rate to the top rate (rho is linear in W^s and in U^s).
    Returns (L, [dW^s], [dU^s])."""
    F = cfg.sample_rate
    chain = rate_chain(bank, F)
    ranges = level_ranges(chain, t_lo, t_hi, cfg.n_up)
    mixing = [np.asarray(s.mixing, np.float64) for s in bank.slices]
    rho = snr_series(x, bank, cfg, t_lo, t_hi, mixing=mixing)
    R = rho - target
    L = float(np.sum(R * R))
    dW, dU = [], []
    for s, W in zip(bank.slices, mixing):
        j = chain.index(int(s.rate))
        lo, hi = ranges[j]
        D = F // s.rate
        N = s.n_taps
        d_lo = lo - s.delay - (N - 1)
        d = downsample(x, D, d_lo, hi - s.delay, cfg.n_down)
        y = correlate(np.asarray(s.basis, np.float64), d, d_lo, s.delay, lo, hi)
        yhat = _upsample_to_top(y, chain, ranges, j, cfg.n_up)
        dW.append(2.0 * R @ yhat.T)
        g = _adjoint_to_level(R, chain, ranges, j, cfg.n_up)
        dy = 2.0 * W.T @ g
        H = sliding_window_view(d, N)          # H[i, n] = d[lo + i - delay - N + 1 + n]
        dU.append(dy @ H)
    return L, dW, dU


def loss_only(x: np.ndarray, bank, target: np.ndarray, cfg: OracleConfig, t_lo: int, t_hi: int) -> float:
    mixing = [np.asarray(s.mixing, np.float64) for s in bank.slices]
    R = snr_series(x, bank, cfg, t_lo, t_hi, mixing=mixing) - target
    return float(np.sum(R * R))


def direct_bank(bank):
    """The multirate-direct bank: every slice at full rank (U^s = H^s,
    W^s = I), from the uncompressed slice templates."""
    from types import SimpleNamespace
    sl = [SimpleNamespace(rate=s.rate, delay=s.delay, basis=H, mixing=np.eye(H.shape[0]), n_taps=H.shape[1],
                          n_basis=H.shape[0]) for s, H in zip(bank.slices, bank.templates)]
    return SimpleNamespace(n_templates=bank.n_templates, slices=sl)


# ---------------------------------------------------------------------------
# Re-orthonormalisation of refined bases (CholeskyQR2, float64)
# ---------------------------------------------------------------------------

def cholesky_qr2(U: np.ndarray, W: np.ndarray):
    """U^T = Q R with Q orthonormal columns, by two CholeskyQR passes:
    G = U U^T = R^T R, U <- R^-T U, W <- W R^T.  W U is unchanged."""
    for _ in range(2):
        G = U @ U.T
        C = np.linalg.cholesky(G)          # G = C C^T, C = R^T lower triangular
        U = np.linalg.solve(C, U)          # R^-T U
        W = W @ C                          # W R^T
    return U, W


# ---------------------------------------------------------------------------
# Signal-consistency statistic xi^2 (Sec. II.D.2)
# ---------------------------------------------------------------------------

def template_autocorrelation(h: np.ndarray, half_width: int) -> np.ndarray:
    """R(t) for t = -half_width..half_width (index t + half_width) of the
    complex templates h [..., n] in tau order, normalised to R(0) = 1
    (reading R20): R(t) = sum_j h[j] conj h[j - t] / sum_j |h[j]|^2."""
    h = np.asarray(h, np.complex128)
    n = h.shape[-1]
    power = np.sum(np.abs(h) ** 2, axis=-1)
    out = np.zeros(h.shape[:-1] + (2 * half_width + 1,), np.complex128)
    for t in range(-half_width, half_width + 1):
        if abs(t) >= n:
            continue
        if t >= 0:                                   # j = t .. n-1
            c = np.sum(h[..., t:] * np.conj(h[..., :n - t]), axis=-1)
        else:                                        # j = 0 .. n-1+t
            c = np.sum(h[..., :n + t] * np.conj(h[..., -t:]), axis=-1)
        out[..., t + half_width] = c / power
    return out


def xi2(z: np.ndarray, t_peak: np.ndarray, R: np.ndarray) -> np.ndarray:
    """xi^2 of Sec. II.D.2 for every row of z (complex [K, T], the SNR series
    around the triggers), at index t_peak[k] of row k, with the
    autocorrelation R [K, A] of that row's template (A odd):

        num = sum_{t=-delta}^{delta} |z(t_p + t) - z(t_p) R(t)|^2
        den = sum_{t=-delta}^{delta} (2 - 2 |R(t)|^2)

    and xi^2 = num / den (reading R21: samples, not integrals; indices
    t_p + t outside [0, T) are left out of both sums)."""
    z = np.asarray(z, np.complex128)
    R = np.asarray(R, np.complex128)
    K, T = z.shape
    A = R.shape[1]
    assert A % 2 == 1 and R.shape[0] == K
    delta = (A - 1) // 2
    rows = np.arange(K)[:, None]
    idx = np.asarray(t_peak, np.int64)[:, None] + np.arange(-delta, delta + 1)[None, :]
    have = (idx >= 0) & (idx < T)
    zt = np.where(have, z[rows, np.clip(idx, 0, T - 1)], 0.0)
    z0 = z[np.arange(K), np.asarray(t_peak, np.int64)][:, None]
    num = np.sum(np.where(have, np.abs(zt - z0 * R) ** 2, 0.0), axis=1)
    den = np.sum(np.where(have, 2.0 - 2.0 * np.abs(R) ** 2, 0.0), axis=1)
    return num / den


# ---------------------------------------------------------------------------
# Overlapping trigger windows, coincidence, clustering (Sec. II.D.3-4)
# ---------------------------------------------------------------------------

def window_trigger(z_prev: Optional[np.ndarray], z_cur: np.ndarray, overlap: int,
                   threshold: float = SNR_THRESHOLD) -> Peaks:
    """Trigger per template over window k = the last `overlap` samples of
    stride k-1 followed by stride k (reading R23; z_prev None: the first,
    shortened window).  Index relative to the start of stride k."""
    if z_prev is None or overlap == 0:
        return window_peaks(z_cur, threshold)
    w = np.concatenate([z_prev[:, z_prev.shape[1] - overlap:], z_cur], axis=1)
    p = window_peaks(w, threshold)
    return Peaks(p.snr, p.index - overlap, p.value, p.above)


@dataclass
class Event:
    template: int          # -1: no coincident event in the sub-bank
    network_snr: float
    det_mask: int          # detectors held by the event


def coincident_events(snr: np.ndarray, index: np.ndarray, above: np.ndarray,
                      window: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Per template (columns of the [n_det, M] trigger arrays), the network
    SNR^2 (float32, summed in detector order) and detector mask of its best
    coincident event (reading R24); 0 and 0 where there is none."""
    n_det, M = snr.shape
    best2 = np.zeros(M, np.float32)
    best_mask = np.zeros(M, np.int64)
    for m in range(M):
        for a in range(n_det):
            if not above[a, m]:
                continue
            held = [d for d in range(n_det)
                    if above[d, m] and (d == a or abs(int(index[d, m]) - int(index[a, m])) <= window[a, d])]
            if len(held) < 2:
                continue
            s2 = np.float32(0.0)
            for d in held:
                s2 = np.float32(s2 + np.float32(snr[d, m]) * np.float32(snr[d, m]))
            if s2 > best2[m]:
                best2[m] = s2
                best_mask[m] = sum(1 << d for d in held)
    return best2, best_mask


def cluster(best2: np.ndarray, mask: np.ndarray) -> Event:
    """One event per sub-bank and window (reading R25): the largest network
    SNR, lowest template on ties."""
    if not np.any(mask):
        return Event(-1, 0.0, 0)
    cand = np.where(mask != 0)[0]
    m = int(cand[np.argmax(best2[cand])])          # argmax takes the first maximum
    return Event(m, float(np.sqrt(np.float32(best2[m]), dtype=np.float32)), int(mask[m]))


# ---------------------------------------------------------------------------
# PSD estimation and whitening with frequency-domain downsampling (Sec. II.B.2)
# ---------------------------------------------------------------------------

def median_bias(c: int) -> float:
    """beta_c = exp(E[log median of c iid unit exponentials] + gamma) for odd
    c (reading R27): the median of c chi^2_2 bins over their geometric mean.
    The median is the order statistic k = (c+1)/2 of c exponentials; its
    density is integrated numerically (SciPy's quad)."""
    from scipy import integrate
    from scipy.special import comb
    assert c % 2 == 1
    k = (c + 1) // 2
    dens = lambda x: comb(c, k) * k * (-np.expm1(-x)) ** (k - 1) * np.exp(-x * (c - k + 1))
    e_log = integrate.quad(lambda x: np.log(x) * dens(x), 0, np.inf, limit=400, epsabs=1e-13, epsrel=1e-13)[0]
    return float(np.exp(e_log + np.euler_gamma))


class Whitener:
    """Streaming PSD estimation and whitening of one detector (Sec. II.B.2,
    readings R26-R28), float64.  push() takes H = N/2 - Z new input samples
    and returns H / D whitened output samples."""

    def __init__(self, n: int, z: int, d: int = 1, n_med: int = 7, n_avg: int = 64):
        assert n & (n - 1) == 0 and 0 <= z <= n // 4 and n % d == 0 and z % d == 0 and n_med % 2 == 1
        self.n, self.z, self.d, self.n_med, self.n_avg = n, z, d, n_med, n_avg
        self.h = n // 2 - z
        assert self.h % d == 0
        self.n_out, self.h_out, self.z_out = n // d, self.h // d, z // d
        self.k_out = self.n_out // 2 + 1
        m = np.arange(2 * self.h)
        self.hann = np.sin(np.pi * m / (2 * self.h)) ** 2
        self.w2 = float(np.sum(self.hann ** 2))
        tk = np.ones(self.n_out)
        if self.z_out > 0:
            r = 0.5 * (1.0 - np.cos(np.pi * np.arange(self.z_out) / self.z_out))
            tk[:self.z_out] = r
            tk[self.n_out - self.z_out:] = r[::-1]
        self.tukey = tk
        self.beta = {c: median_bias(c) for c in range(1, n_med + 1, 2)}
        self.seg = np.zeros(2 * self.h)
        self.acc = np.zeros(self.n_out)
        self.recent: List[np.ndarray] = []
        self.log_geo = np.zeros(self.k_out)
        self.blocks = 0

    def running_median(self) -> Tuple[np.ndarray, int]:
        """Per bin, the median of the most recent c instantaneous estimates,
        c = the largest odd count <= min(blocks seen, n_med) (reading R27),
        and c."""
        c = min(self.blocks, self.n_med)
        c -= 1 - c % 2
        return np.median(np.stack(self.recent[-c:]), axis=0), c

    @property
    def psd(self) -> np.ndarray:
        return np.exp(self.log_geo) * np.exp(np.euler_gamma)

    def push(self, x: np.ndarray, gap: bool = False) -> np.ndarray:
        x = np.asarray(x, np.float64)
        assert x.shape == (self.h,)
        self.seg = np.concatenate([self.seg[self.h:], np.zeros(self.h) if gap else x])
        if not gap:
            blk = np.zeros(self.n)
            blk[self.z:self.z + 2 * self.h] = self.hann * self.seg
            X = np.fft.rfft(blk)[:self.k_out]                       # frequency-domain downsampling
            P = (X.real ** 2 + X.imag ** 2) / self.w2                # instantaneous PSD
            self.recent = (self.recent + [P])[-self.n_med:]
            self.blocks += 1
            med, c = self.running_median()
            obs = np.log(med / self.beta[c])
            self.log_geo += (obs - self.log_geo) / min(self.blocks, self.n_avg)
            Y = X / np.sqrt(self.d * self.psd)
            y = np.fft.irfft(Y, self.n_out)
            self.acc += self.tukey * y
        out = self.acc[:self.h_out].copy()
        self.acc = np.concatenate([self.acc[self.h_out:], np.zeros(self.h_out)])
        return out


# ---------------------------------------------------------------------------
# FP8 basis values for quantisation-aware refinement (extension; reading 19)
# ---------------------------------------------------------------------------

def e4m3_round(x: np.ndarray) -> np.ndarray:
    """Nearest OCP e4m3 value (4 exponent bits, bias 7, 3 mantissa bits,
    subnormals below 2^-6, largest finite 448), ties to the even mantissa;
    |x| <= 448.  In a binade [2^e, 2^(e+1)) the spacing is 2^(e-3); below
    2^-6 it is 2^-9."""
    x = np.asarray(x, np.float64)
    a = np.abs(x)
    e = np.clip(np.floor(np.log2(np.where(a > 0, a, 1.0))), -6, 8)
    q = 2.0 ** (e - 3)
    return np.sign(x) * np.round(a / q) * q          # np.round: half to even


def quantize_fp8_rows(U: np.ndarray) -> np.ndarray:
    """The basis values the FP8 form correlates with, as float64: per row a
    power-of-two scale 2^e, e = floor(log2(448 / max|u|)), then e4m3 of the
    float32-rounded u 2^e (the precision the GPU rounds from), times 2^-e."""
    U = np.asarray(U, np.float64)
    mx = np.abs(U).max(axis=1)
    e = np.where(mx > 0, np.floor(np.log2(448.0 / np.where(mx > 0, mx, 1.0))), 0.0)
    s = 2.0 ** e
    x32 = (U * s[:, None]).astype(np.float32).astype(np.float64)
    return e4m3_round(x32) / s[:, None]


# ---------------------------------------------------------------------------
# SVD bank construction (Sec. II.C.1)
# ---------------------------------------------------------------------------

def svd_truncate(H: np.ndarray, L: int) -> Tuple[np.ndarray, np.ndarray]:
    """Rank-L truncated SVD of a slice's template matrix H [2M, N] (NumPy's
    SVD as the library step): basis rows U = the first L right singular
    vectors, mixing W = (left singular vectors x singular values)[:, :L], so
    W U is the best rank-L approximation of H."""
    Ul, sv, Vt = np.linalg.svd(np.asarray(H, np.float64), full_matrices=False)
    return Vt[:L].copy(), Ul[:, :L] * sv[:L]
