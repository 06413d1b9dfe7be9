"""Pins of the oracle's overlapping trigger windows, coincidence and
clustering (Sec. II.D.3-4, readings R23-R25), CPU only.

* windows: overlap 0 is the per-stride trigger; a peak inside the overlap is
  seen by both windows at the same absolute time; over a long series the
  windows' maxima include the global maximum and every sample is covered;
* coincidence: two detectors reduce to the closed form (both above the
  threshold and |dt| <= w, network SNR sqrt(rho1^2 + rho2^2)); an unbounded
  window holds every detector above the threshold; a zero window only
  identical times; one detector never makes an event; results are invariant
  under a common time shift and equivariant under a detector permutation;
* clustering: the largest network SNR, lowest template on ties, none when no
  template has an event;
* end to end through the oracle filter: a chirp injected into two detectors
  10 ms apart gives a two-detector event at the injected template, and none
  when the delay exceeds the window.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import lloid as O


def _rand_triggers(g, n_det, M, T=4096):
    snr = g.uniform(2.0, 9.0, (n_det, M)).astype(np.float32)
    idx = g.integers(-100, T, (n_det, M))
    return snr, idx, snr >= O.SNR_THRESHOLD


def test_window_without_overlap_is_the_stride_trigger():
    g = synth.rng_for(94, synth.PURPOSE_NOISE, 0)
    z0, z1 = (g.standard_normal((5, 512)) + 1j * g.standard_normal((5, 512)) for _ in range(2))
    a, b = O.window_trigger(z0, z1, 0), O.window_peaks(z1)
    assert np.array_equal(a.index, b.index) and np.array_equal(a.snr, b.snr)
    c = O.window_trigger(None, z1, 40)
    assert np.array_equal(c.index, b.index)


def test_peak_in_the_overlap_is_seen_by_both_windows():
    g = synth.rng_for(94, synth.PURPOSE_NOISE, 1)
    F, Ov = 512, 60
    z = g.standard_normal((3, 3 * F)) + 1j * g.standard_normal((3, 3 * F))
    z[:, 2 * F - 7] = 50.0                       # 7 samples before stride 2 starts
    w1 = O.window_trigger(z[:, :F], z[:, F:2 * F], Ov)
    w2 = O.window_trigger(z[:, F:2 * F], z[:, 2 * F:], Ov)
    assert np.all(w1.index == F - 7) and np.all(w2.index == -7)
    assert np.all(w1.snr == 50.0) and np.all(w2.snr == 50.0)


def test_windows_cover_the_series_and_keep_the_global_maximum():
    g = synth.rng_for(94, synth.PURPOSE_NOISE, 2)
    F, Ov, K = 256, 33, 9
    z = g.standard_normal((4, K * F)) + 1j * g.standard_normal((4, K * F))
    seen = np.zeros(K * F, int)
    best = np.full(4, -1.0)
    for k in range(K):
        w = O.window_trigger(z[:, (k - 1) * F:k * F] if k else None, z[:, k * F:(k + 1) * F], Ov)
        lo = max(k * F - Ov, 0)
        seen[lo:(k + 1) * F] += 1
        best = np.maximum(best, w.snr)
        assert np.allclose(np.abs(z[np.arange(4), k * F + w.index]), w.snr)
    assert np.all(seen >= 1) and np.all(seen <= 2) and seen.sum() == K * F + (K - 1) * Ov
    assert np.allclose(best, np.abs(z).max(axis=1))


def test_two_detectors_closed_form():
    g = synth.rng_for(94, synth.PURPOSE_STRUCT, 3)
    snr, idx, above = _rand_triggers(g, 2, 400)
    w = np.array([[0, 40], [40, 0]])
    best2, mask = O.coincident_events(snr, idx, above, w)
    hit = above[0] & above[1] & (np.abs(idx[0] - idx[1]) <= 40)
    assert np.array_equal(mask != 0, hit) and np.all(mask[hit] == 3)
    ref = snr[0].astype(np.float64) ** 2 + snr[1].astype(np.float64) ** 2
    assert np.allclose(best2[hit], ref[hit], rtol=1e-6) and np.all(best2[~hit] == 0)


def test_unbounded_and_zero_windows():
    g = synth.rng_for(94, synth.PURPOSE_STRUCT, 4)
    snr, idx, above = _rand_triggers(g, 4, 300)
    big = np.full((4, 4), 10 ** 9)
    best2, mask = O.coincident_events(snr, idx, above, big)
    n_above = above.sum(axis=0)
    ev = n_above >= 2
    assert np.all((mask != 0) == ev)
    full = np.sum(np.where(above, snr.astype(np.float64) ** 2, 0.0), axis=0)
    assert np.allclose(best2[ev], full[ev], rtol=1e-6)
    assert np.all(mask[ev] == np.sum(np.where(above, 1 << np.arange(4)[:, None], 0), axis=0)[ev])
    idx2 = idx.copy()
    idx2[1] = idx2[0]                              # detectors 0 and 1 simultaneous, others random
    best2, mask = O.coincident_events(snr, idx2, above, np.zeros((4, 4), int))
    pair = above[0] & above[1]
    assert np.all((mask[pair] & 3) == 3)


def test_one_detector_never_makes_an_event():
    snr = np.full((1, 10), 9.0, np.float32)
    best2, mask = O.coincident_events(snr, np.zeros((1, 10), int), snr >= 4, np.zeros((1, 1), int))
    assert not mask.any() and O.cluster(best2, mask).template == -1


def test_shift_invariance_and_detector_permutation():
    g = synth.rng_for(94, synth.PURPOSE_STRUCT, 5)
    snr, idx, above = _rand_triggers(g, 3, 500)
    w = np.array([[0, 41, 113], [41, 0, 110], [113, 110, 0]])
    b0, m0 = O.coincident_events(snr, idx, above, w)
    b1, m1 = O.coincident_events(snr, idx + 777, above, w)
    assert np.array_equal(b0, b1) and np.array_equal(m0, m1)
    for perm in itertools.permutations(range(3)):
        p = np.array(perm)
        bp, mp = O.coincident_events(snr[p], idx[p], above[p], w[np.ix_(p, p)])
        back = np.zeros_like(m0)
        for new, old in enumerate(perm):
            back |= ((mp >> new) & 1) << old
        assert np.array_equal(back, m0)
        assert np.allclose(bp, b0, rtol=1e-6)


def test_cluster_picks_the_largest_lowest_template_on_ties():
    best2 = np.array([0, 50, 80, 80, 10], np.float32)
    mask = np.array([0, 3, 3, 3, 3])
    e = O.cluster(best2, mask)
    assert e.template == 2 and e.det_mask == 3 and abs(e.network_snr - np.sqrt(80)) < 1e-5
    assert O.cluster(best2, np.zeros(5, int)).template == -1


@pytest.mark.parametrize("delay_ms,expect", [(10.0, True), (40.0, False)])
def test_injected_signal_is_a_coincident_event(delay_ms, expect):
    F = 4096
    bank = synth.chirp_bank(F, 16, 30.0, (1.0, 2.0), [(4096, 0.0, 1024, 24), (1024, 0.25, 1800, 30)],
                            seed=[94, 1, 0])
    x = synth.gaussian_strain(94, 2, 3 * F)
    dt = int(round(delay_ms * 1e-3 * F))
    synth.inject(x, F, bank, synth.Injection(0, 9, 0, 2 * F + 1000, 14.0))
    synth.inject(x, F, bank, synth.Injection(0, 9, 1, 2 * F + 1000 + dt, 12.0))
    Ov = int(round((0.0273 + 0.005) * F))
    w = np.full((2, 2), Ov)
    cfg = O.OracleConfig(F)
    trig = []
    for d in range(2):
        z, _ = O.lloid_filter(x[d], bank, cfg, n_strides=2, first_stride=1)
        trig.append(O.window_trigger(z[:, :F], z[:, F:], Ov))
    snr = np.stack([t.snr for t in trig]).astype(np.float32)
    idx = np.stack([t.index for t in trig])
    above = np.stack([t.above for t in trig])
    e = O.cluster(*O.coincident_events(snr, idx, above, w))
    assert abs(idx[0, 9] - 1000) <= 8 and abs(idx[1, 9] - 1000 - dt) <= 8   # ~2 ms timing in noise
    if expect:
        assert e.template == 9 and e.det_mask == 3
        assert abs(e.network_snr - np.hypot(snr[0, 9], snr[1, 9])) < 1e-4
    else:
        assert e.template != 9 or e.det_mask != 3


def test_window_edge_is_inclusive():
    snr = np.full((2, 3), 6.0, np.float32)
    idx = np.array([[100, 100, 100], [140, 141, 60]])
    best2, mask = O.coincident_events(snr, idx, snr >= 4, np.array([[0, 40], [40, 0]]))
    assert list(mask) == [3, 0, 3]
