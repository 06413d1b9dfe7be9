"""Pins of the oracle's PSD estimation and whitening with frequency-domain
downsampling (Sec. II.B.2, readings R26-R28), CPU only.

* the periodic Hann window sums to one at hop H; the Tukey window is one
  over the segment;
* the median bias beta_1 = 1 exactly (E log of a unit exponential is
  -gamma) and beta_3,5,7 match NumPy medians of exponential samples;
* white noise of any level: the PSD converges to its variance and the
  output has unit variance and zero mean, at D = 1 and D = 4;
* coloured (AR(1)) noise: the output spectrum is flat where the input's
  spans two decades;
* downsampling in the frequency domain: a strong tone above the output
  Nyquist frequency does not alias into the output;
* timing: an impulse at input time t comes out at output time t / D
  (latency N/2 as stated), and a run of gap pushes drains the output to
  exact zeros without touching the PSD;
* steady state in white noise: the mean over bins and pushes of
  log(PSD / sigma^2) is zero within 4 standard errors (about 0.0025), which
  pins the median count c and its bias factor beta_c together: beta_5 in
  place of beta_7 is a 0.016 bias in the log;
* planted slips (no e^gamma, symmetric instead of periodic Hann, beta of
  the next smaller count, a median over one estimate too few) break a pin.
"""
import numpy as np
import pytest

import synth
from oracle import lloid as O


def _run(w, x, pushes):
    return np.concatenate([w.push(x[i * w.h:(i + 1) * w.h]) for i in range(pushes)])


def test_hann_sums_to_one_and_tukey_is_flat_over_the_segment():
    w = O.Whitener(2048, 256, d=2)
    h = w.h
    tot = w.hann[:h] + w.hann[h:]
    assert np.allclose(tot, 1.0, atol=1e-15)
    assert np.all(w.tukey[w.z_out:w.n_out - w.z_out] == 1.0) and w.tukey[0] == 0.0


def test_median_bias():
    assert abs(O.median_bias(1) - 1.0) < 1e-12
    g = synth.rng_for(92, synth.PURPOSE_NOISE, 0)
    for c in (3, 5, 7):
        e = np.log(np.median(g.exponential(size=(400000, c)), axis=1))
        est = np.exp(e.mean() + np.euler_gamma)
        se = e.std() / np.sqrt(len(e)) * est
        assert abs(est - O.median_bias(c)) < 4 * se, (c, est, O.median_bias(c))


@pytest.mark.parametrize("sigma,d", [(1.0, 1), (3.0, 4), (0.01, 4)])
def test_white_noise_gives_unit_variance(sigma, d):
    w = O.Whitener(4096, 512, d=d)
    x = sigma * synth.rng_for(92, synth.PURPOSE_NOISE, 1).standard_normal(300 * w.h)
    out = _run(w, x, 300)[40 * w.h_out:]
    assert abs(out.std() - 1.0) < 0.03 and abs(out.mean()) < 0.02
    assert abs(np.median(w.psd[1:-1]) / sigma ** 2 - 1.0) < 0.05


def test_coloured_noise_is_whitened():
    w = O.Whitener(4096, 512, d=2)
    e = synth.rng_for(92, synth.PURPOSE_NOISE, 2).standard_normal(300 * w.h)
    x = np.zeros_like(e)
    for i in range(1, len(e)):                     # AR(1): strongly red
        x[i] = 0.95 * x[i - 1] + e[i]
    out = _run(w, x, 300)[40 * w.h_out:]

    def band_ratio(v, n):
        seg = v[:len(v) // n * n].reshape(-1, n)
        p = np.mean(np.abs(np.fft.rfft(seg * np.hanning(n), axis=1)) ** 2, axis=0)
        k = len(p)
        return p[1:k // 8].mean() / p[k // 2:7 * k // 8].mean()

    assert band_ratio(x, 1024) > 100.0
    assert abs(band_ratio(out, 1024) - 1.0) < 0.1
    assert abs(out.std() - 1.0) < 0.05


def test_tone_above_the_output_nyquist_does_not_alias():
    w = O.Whitener(4096, 512, d=4)
    n = 200 * w.h
    t = np.arange(n)
    g = synth.rng_for(92, synth.PURPOSE_NOISE, 3)
    f = 0.3                                        # cycles/sample: above the output Nyquist 0.125
    x = g.standard_normal(n) + 50.0 * np.sin(2 * np.pi * f * t)
    out = _run(w, x, 200)[40 * w.h_out:]
    assert abs(out.std() - 1.0) < 0.03             # a naive decimation would alias the tone in


def test_impulse_timing_and_gap_drain():
    w = O.Whitener(2048, 256, d=2)
    g = synth.rng_for(92, synth.PURPOSE_NOISE, 4)
    pushes = 60
    x = g.standard_normal(pushes * w.h)
    t0 = 40 * w.h + 123
    x[t0] += 400.0
    out = _run(w, x, pushes)
    # push i (1-based) outputs input times [iH - 2H - Z, iH - H - Z) at rate 1/D
    first_time = w.h - 2 * w.h - w.z                  # input time of output sample 0
    peak = int(np.argmax(np.abs(out)))
    assert abs(first_time + peak * w.d - t0) <= w.d
    psd = w.psd.copy()
    drained = [w.push(np.zeros(w.h), gap=True) for _ in range(4)]
    assert np.array_equal(w.psd, psd)
    assert np.all(drained[-1] == 0.0) and np.any(drained[0] != 0.0)


@pytest.mark.parametrize("slip", ["no_euler_gamma", "symmetric_hann"])
def test_planted_slip_breaks_a_pin(monkeypatch, slip):
    w = O.Whitener(4096, 512, d=1)
    if slip == "no_euler_gamma":
        monkeypatch.setattr(O.Whitener, "psd", property(lambda self: np.exp(self.log_geo)))
        x = synth.rng_for(92, synth.PURPOSE_NOISE, 5).standard_normal(200 * w.h)
        out = _run(w, x, 200)[40 * w.h_out:]
        assert abs(out.std() - 1.0) > 0.2
    else:
        w.hann = np.hanning(2 * w.h)
        assert not np.allclose(w.hann[:w.h] + w.hann[w.h:], 1.0, atol=1e-6)


STEADY_N, STEADY_Z, STEADY_PUSHES, STEADY_BURN = 1 << 16, 1 << 13, 600, 400


def _steady_log_psd(w, sigma, seed):
    """Mean over interior bins and over pushes STEADY_BURN.. of log(PSD /
    sigma^2) in white noise, and its standard error from 64 groups of
    adjacent bins (bins further apart than the Hann window's main lobe are
    nearly independent; the groups average over hundreds of them).

    Expectation: with beta_c correct, log(median of c / beta_c) averages
    log sigma^2 - gamma for every odd c, so log PSD averages log sigma^2.
    The first block (half zeros) biases the running average low by about
    log(2) / n_avg; after STEADY_BURN pushes its weight has decayed by
    (1 - 1/n_avg)^(STEADY_BURN - n_avg) < 0.006, a bias below 1e-4."""
    x = sigma * synth.rng_for(93, synth.PURPOSE_NOISE, seed).standard_normal(STEADY_PUSHES * w.h)
    acc = np.zeros(w.k_out - 2)
    for i in range(STEADY_PUSHES):
        w.push(x[i * w.h:(i + 1) * w.h])
        if i >= STEADY_BURN:
            acc += np.log(w.psd[1:-1] / sigma ** 2)
    per_bin = acc / (STEADY_PUSHES - STEADY_BURN)
    k = per_bin.shape[0] // 64 * 64
    groups = per_bin[:k].reshape(64, -1).mean(axis=1)
    return float(per_bin.mean()), float(groups.std(ddof=1) / np.sqrt(64))


def _beta_of_smaller_count(w):
    b = dict(w.beta)
    w.beta = {c: (b[c - 2] if c >= 3 else b[c]) for c in b}


def _median_over_one_fewer(w):
    """Median of the most recent c - 1 estimates (an even count: NumPy
    averages the middle two) divided by beta_c."""
    def slipped(self):
        c = min(self.blocks, self.n_med)
        c -= 1 - c % 2
        n = max(c - 1, 1)
        return np.median(np.stack(self.recent[-n:]), axis=0), c
    w.running_median = slipped.__get__(w)


def test_steady_state_psd_is_unbiased():
    w = O.Whitener(STEADY_N, STEADY_Z, d=1)
    mean, se = _steady_log_psd(w, 2.0, 0)
    assert abs(mean) < 4 * se + 1e-4, (mean, se)
    assert se < 2e-3


@pytest.mark.parametrize("slip", ["beta_of_smaller_count", "median_over_one_fewer"])
def test_psd_bookkeeping_slip_breaks_the_steady_state_pin(slip):
    w = O.Whitener(STEADY_N, STEADY_Z, d=1)
    if slip == "beta_of_smaller_count":
        _beta_of_smaller_count(w)
    else:
        _median_over_one_fewer(w)
    mean, se = _steady_log_psd(w, 2.0, 0)
    assert abs(mean) > 4 * se + 1e-4, (mean, se)
