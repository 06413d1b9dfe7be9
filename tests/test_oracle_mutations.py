"""Planted mistakes in the oracle (CPU only) must make a pin fail.

Each case patches one step of the oracle with a plausible slip and checks
that the direct-filter pins (single-rate chain, band-limited multirate
chain) no longer hold."""
import numpy as np
import pytest

import synth
from oracle import lloid as O

F = 1024
TINY3 = [(1024, 0.0, 128, 16), (512, 0.125, 192, 16), (256, 0.5, 384, 16)]


def _multirate_error(x):
    bank = synth.burst_bank(F, 8, TINY3, seed=[9, 1, 0])
    rho = O.snr_series(x, bank, O.OracleConfig(F, normalize=False), 3 * F, 5 * F)
    ref = O.brute_force(x, synth.burst_full_rate(bank, F), 3 * F, 5 * F)
    return np.abs(rho - ref).max() / np.abs(ref).max()


def _single_rate_error(x):
    sl = [(1024, 0.0, 256, 6), (1024, 0.25, 700, 9)]
    bank = synth.chirp_bank(F, 8, 20.0, (0.5, 0.9), sl, seed=[9, 1, 0])
    rho = O.snr_series(x, bank, O.OracleConfig(F), 3 * F, 4 * F)
    ref = O.brute_force(x, O.concatenated_filters(bank, F, O.normalized_mixing(bank)), 3 * F, 4 * F)
    return np.abs(rho - ref).max() / np.abs(ref).max()


def _slip_delay(orig):
    def f(U, d, d_lo, delay, q_lo, q_hi):
        late = np.concatenate([[0.0], d[:-1]])              # every read one sample late
        return orig(U, late, d_lo, delay, q_lo, q_hi)
    return f


def _slip_gain(orig):
    def f(x, D, m_lo, m_hi, n_down=O.N_DOWN):
        return orig(x, D, m_lo, m_hi, n_down) / (np.sqrt(D) if D > 1 else 1.0)
    return f


def _slip_upsample_phase(orig):
    def f(a, a_lo, p, i_lo, i_hi, n_up=O.N_UP):
        late = np.concatenate([np.zeros((a.shape[0], 1)), a[:, :-1]], axis=1)
        return orig(late, a_lo, p, i_lo, i_hi, n_up)        # interpolates one input late
    return f


def _slip_reversed_taps(orig):
    def f(U, d, d_lo, delay, q_lo, q_hi):
        return orig(np.ascontiguousarray(U[:, ::-1]), d, d_lo, delay, q_lo, q_hi)
    return f


@pytest.mark.parametrize("name,slip,which", [
    ("correlate", _slip_delay, "both"),
    ("downsample", _slip_gain, "multirate"),
    ("upsample", _slip_upsample_phase, "multirate"),
    ("correlate", _slip_reversed_taps, "both"),
])
def test_planted_mistake_breaks_a_pin(monkeypatch, name, slip, which):
    x = synth.gaussian_strain(99, 1, 8 * F)[0]
    assert _multirate_error(x) < 2e-3 and _single_rate_error(x) < 1e-12
    monkeypatch.setattr(O, name, slip(getattr(O, name)))
    if which in ("both", "multirate"):
        assert _multirate_error(x) > 1e-2
    if which == "both":
        assert _single_rate_error(x) > 1e-2
