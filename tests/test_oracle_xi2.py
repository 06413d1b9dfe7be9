"""Pins of the oracle's signal-consistency statistic xi^2 (Sec. II.D.2) and
of the template autocorrelation it uses (readings R20-R22), CPU only.

* the autocorrelation equals the one NumPy's FFT gives (Wiener-Khinchin),
  is Hermitian and has R(0) = 1;
* it is the noise covariance of the filter output: E[z(t) conj z(0)] = 2 R(t)
  over white noise filtered with np.convolve;
* xi^2 vanishes for an SNR series that is exactly z(0) R(t - t_p), and a
  residual e with e(t_p) = 0 adds |e|^2 / den;
* in white noise the numerator's expectation is the denominator: the mean of
  xi^2 at fixed times is 1, also for windows clipped at the data's edge;
* it is invariant under a common phase and scales as |z|^2.
"""
import numpy as np
import pytest

import synth
from oracle import lloid as O

RATE = 1024


def chirp_template(f0=40.0, tc=0.5, rate=RATE):
    """Complex template h = h_cos + i h_sin in tau order, unit-norm parts."""
    n = int(np.ceil(tc * rate)) + 1
    c, s = synth.chirp_pair(np.arange(n) / rate, f0, tc)
    return c / np.linalg.norm(c) + 1j * s / np.linalg.norm(s)


def noise_xi2(h, A, n_real=8, T=1 << 17, clip=None, acf=O.template_autocorrelation, xi2=O.xi2):
    """xi^2 at fixed times (not peaks) of white noise filtered by h, windows
    spaced so that samples are nearly independent.  clip: keep only this
    many samples before the evaluation time (an edge-clipped window)."""
    d = (A - 1) // 2
    R = acf(h, d)
    n = len(h)
    out = []
    for seed in range(n_real):
        x = synth.rng_for(95, synth.PURPOSE_NOISE, seed).standard_normal(T)
        z = np.convolve(x, h)[:T]                      # z[t] = sum_j h[j] x[t - j]
        t0 = np.arange(n - 1 + d, T - d, A + n)
        before = d if clip is None else clip
        win = np.stack([z[t - before:t + d + 1] for t in t0])
        out.append(xi2(win, np.full(len(t0), before), np.tile(R, (len(t0), 1))))
    return np.concatenate(out)


def test_autocorrelation_matches_fft():
    h = chirp_template()
    d = 300
    R = O.template_autocorrelation(h, d)
    N = 4 * len(h)
    H = np.fft.fft(h, N)
    c = np.fft.ifft(H * np.conj(H))                   # c[t] = sum_j h[j] conj h[j - t], circular
    ref = np.concatenate([c[N - d:], c[:d + 1]]) / np.sum(np.abs(h) ** 2)
    assert np.abs(R - ref).max() < 1e-12
    assert abs(R[d] - 1) < 1e-14
    assert np.abs(R - np.conj(R[::-1])).max() < 1e-14    # R(-t) = conj R(t)
    assert np.all(np.abs(R) <= 1 + 1e-12)                # Cauchy-Schwarz


def test_autocorrelation_beyond_the_template_is_zero():
    h = chirp_template(tc=0.05)                          # 52 taps
    R = O.template_autocorrelation(h, 80)
    assert np.all(R[:80 - 51] == 0) and np.all(R[80 + 52:] == 0)


def test_autocorrelation_is_the_noise_covariance():
    h = chirp_template()
    d = 60
    R = O.template_autocorrelation(h, d)
    acc = np.zeros(2 * d + 1, complex)
    cnt = 0
    for seed in range(4):
        x = synth.rng_for(95, synth.PURPOSE_NOISE, 100 + seed).standard_normal(1 << 17)
        z = np.convolve(x, h)[len(h):1 << 17]
        t = np.arange(d, len(z) - d)
        for k in range(-d, d + 1):
            acc[k + d] += np.sum(z[t + k] * np.conj(z[t]))
        cnt += len(t)
    est = acc / cnt / 2.0
    # each lag's estimate averages ~5e5 products of correlated samples
    assert np.abs(est - R).max() < 0.02


def test_xi2_is_zero_for_an_exact_template_response():
    g = synth.rng_for(95, synth.PURPOSE_STRUCT, 1)
    h = chirp_template()
    A = 351
    d = (A - 1) // 2
    R = O.template_autocorrelation(h, d)
    T = 1000
    for tp in (0, 5, 175, 500, 824, 999):
        z = g.standard_normal(T) + 1j * g.standard_normal(T)
        amp = 7.0 * np.exp(1j * g.uniform(0, 2 * np.pi))
        for t in range(-d, d + 1):
            if 0 <= tp + t < T:
                z[tp + t] = amp * R[t + d]
        v = O.xi2(z[None], np.array([tp]), R[None])[0]
        assert abs(v) < 1e-20


def test_xi2_residual_adds_its_energy():
    g = synth.rng_for(95, synth.PURPOSE_STRUCT, 2)
    h = chirp_template(f0=60.0, tc=0.3)
    A = 201
    d = 100
    R = O.template_autocorrelation(h, d)
    T = 600
    tp = 300
    e = g.standard_normal(A) + 1j * g.standard_normal(A)
    e[d] = 0.0
    z = np.zeros(T, complex)
    z[tp - d:tp + d + 1] = 5.0 * R + e
    den = np.sum(2.0 - 2.0 * np.abs(R) ** 2)
    v = O.xi2(z[None], np.array([tp]), R[None])[0]
    assert abs(v - np.sum(np.abs(e) ** 2) / den) < 1e-12 * np.sum(np.abs(e) ** 2) / den


@pytest.mark.parametrize("A", [351, 701])
def test_xi2_mean_in_noise_is_one(A):
    v = noise_xi2(chirp_template(), A)
    se = v.std() / np.sqrt(len(v))
    assert abs(v.mean() - 1.0) < 5 * se, (v.mean(), se)


def test_xi2_mean_in_noise_is_one_for_clipped_windows():
    v = noise_xi2(chirp_template(), 351, clip=20)
    se = v.std() / np.sqrt(len(v))
    assert abs(v.mean() - 1.0) < 5 * se, (v.mean(), se)


def test_xi2_phase_invariance_and_scaling():
    g = synth.rng_for(95, synth.PURPOSE_STRUCT, 3)
    h = chirp_template()
    R = O.template_autocorrelation(h, 50)
    z = g.standard_normal((4, 300)) + 1j * g.standard_normal((4, 300))
    tp = np.array([0, 120, 250, 299])
    RR = np.tile(R, (4, 1))
    base = O.xi2(z, tp, RR)
    rot = O.xi2(z * np.exp(1.234j), tp, RR)
    big = O.xi2(3.0 * z, tp, RR)
    assert np.allclose(rot, base, rtol=1e-12) and np.allclose(big, 9.0 * base, rtol=1e-12)


# Planted mistakes: each slip must break one of the pins above.

def _acf_reversed(h, d):
    return O.template_autocorrelation(h, d)[::-1]           # t -> -t, i.e. conj R


def _acf_unnormalised(h, d):
    return O.template_autocorrelation(h, d) * np.sum(np.abs(h) ** 2)   # no division by sum |h|^2


@pytest.mark.parametrize("slip", [_acf_reversed, _acf_unnormalised])
def test_planted_autocorrelation_slip_breaks_the_noise_mean(slip):
    v = noise_xi2(chirp_template(), 351, acf=slip)
    se = v.std() / np.sqrt(len(v))
    assert abs(v.mean() - 1.0) > 10 * se


def test_planted_window_offset_breaks_the_exact_response():
    h = chirp_template()
    d = 175
    R = O.template_autocorrelation(h, d)
    z = np.zeros(1000, complex)
    z[500 - d:500 + d + 1] = 3.0 * R
    assert O.xi2(z[None], np.array([500]), R[None])[0] < 1e-20
    assert O.xi2(z[None], np.array([501]), R[None])[0] > 1e-3
