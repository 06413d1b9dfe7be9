"""Pins of the FP64 oracle against facts fixed outside the oracle itself:
library routines, closed forms, exact special cases, brute force on tiny
banks, invariants.  CPU only."""
import numpy as np
import pytest
import scipy.signal

import synth
from oracle import lloid as O

F = 1024
TINY3 = [(1024, 0.0, 128, 16), (512, 0.125, 192, 16), (256, 0.5, 384, 16)]


@pytest.fixture(scope="module")
def noise():
    return synth.gaussian_strain(99, 1, 8 * F)[0]


# --------------------------------------------------------------- kernels

@pytest.mark.parametrize("f,c", [(2, 64), (4, 128), (16, 512), (4, 32), (8, 64)])
def test_sinc_kernel_is_sinc_times_lanczos_window(f, c):
    """Eq. (sinc): the second factor is the Lanczos window of 2c+1 points."""
    g = O.sinc_windowed_sinc(f, c)
    k = np.arange(2 * c + 1)
    ref = np.sinc((k - c) / f) * scipy.signal.windows.lanczos(2 * c + 1)
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-15)
    assert g[c] == 1.0
    # zeros of the first factor at multiples of f away from the centre
    m = np.arange(1, c // f + 1) * f
    assert np.abs(g[c + m]).max() < 1e-15 and np.abs(g[c - m]).max() < 1e-15


@pytest.mark.parametrize("D", [2, 4, 8, 16, 64])
def test_downsampler_frequency_response(D):
    """Unit DC gain times sqrt(D); flat passband, -6 dB at the new Nyquist
    frequency, < 1e-3 stopband from 1.1x Nyquist (response by scipy.freqz)."""
    g, c = O.downsample_kernel(D)
    nyq = np.pi / D
    w = np.array([0.0, 0.25, 0.5, 0.8, 1.0, 1.1, 1.5, 2.0]) * nyq
    _, H = scipy.signal.freqz(g, worN=w)
    G = np.real(H * np.exp(1j * w * c)) / np.sqrt(D)       # zero-phase response
    assert abs(G[0] - 1) < 1e-14
    assert abs(G[1] - 1) < 2e-6 and abs(G[2] - 1) < 1e-5
    assert abs(G[3] - 1) < 1e-3
    assert abs(G[4] - 0.5) < 1e-5
    assert np.abs(G[5:]).max() < 1e-3
    # the imaginary part vanishes: the kernel is symmetric (zero phase about c)
    assert np.abs(np.imag(H * np.exp(1j * w * c))).max() < 1e-12


def test_downsample_identity_at_D1(noise):
    np.testing.assert_array_equal(O.downsample(noise, 1, 100, 300), noise[100:300])


@pytest.mark.parametrize("D,frac", [(2, 0.3), (4, 0.5), (16, 0.2), (8, 0.9)])
def test_downsample_sinusoid_passthrough(D, frac):
    """cos(w n + phi) decimated is G(w) cos(w D m + phi), G from scipy."""
    g, c = O.downsample_kernel(D)
    w = frac * np.pi / D
    n = np.arange(0, 40 * D * 64)
    x = np.cos(w * n + 0.7)
    m_lo, m_hi = 80, 600
    d = O.downsample(x, D, m_lo, m_hi)
    _, H = scipy.signal.freqz(g, worN=[w])
    G = np.real(H[0] * np.exp(1j * w * c))
    m = np.arange(m_lo, m_hi)
    np.testing.assert_allclose(d, G * np.cos(w * D * m + 0.7), rtol=0, atol=1e-12)


@pytest.mark.parametrize("p", [2, 4, 8])
def test_upsampler_phase0_passthrough_and_interpolation(p):
    """Eq. (upsample): phase-0 outputs are the input samples exactly; other
    phases interpolate a sinusoid below half the input Nyquist frequency to
    the windowed-sinc accuracy (< 1.5e-3)."""
    q = np.arange(-40, 400)
    for frac in (0.1, 0.25, 0.5):
        w = frac * np.pi
        a = np.cos(w * q + 0.3)[None, :]
        out = O.upsample(a, -40, p, 0, 300 * p)[0]
        i = np.arange(300 * p)
        np.testing.assert_array_equal(out[0::p], a[0, 40:340])
        assert np.abs(out - np.cos(w * i / p + 0.3)).max() < 1.5e-3


def test_upsampler_subkernels_sum_to_one():
    """Each polyphase sub-kernel of the interpolator has unit DC gain to
    within the windowed-sinc ripple."""
    for p in (2, 4, 8):
        z = O.polyphase_subkernels(p)
        assert np.abs(z.sum(axis=1) - 1).max() < 2e-3
        assert z.shape == (p, 17)


# --------------------------------------------------------------- bank / SVD

def test_svd_full_rank_reconstruction():
    bank = synth.chirp_bank(F, 8, 20.0, (1.0, 2.0), TINY3, seed=[9, 1, 0], keep_templates=True)
    for s, H in zip(bank.slices, bank.templates):
        assert np.linalg.norm(s.mixing @ s.basis - H) <= 1e-12 * np.linalg.norm(H)
        np.testing.assert_allclose(s.basis @ s.basis.T, np.eye(s.n_basis), atol=1e-12)


# --------------------------------------------------------------- whole chain

def test_single_rate_chain_equals_direct_filter(noise):
    """All slices at the top rate: correlation + mixing + slicing + delays
    reproduce the direct top-rate correlation with the concatenated filters
    W~U (truncated bank, so the filters are not the chirps themselves)."""
    sl = [(1024, 0.0, 256, 6), (1024, 0.25, 700, 9), (1024, 0.25 + 700 / 1024, 1100, 12)]
    bank = synth.chirp_bank(F, 8, 20.0, (1.0, 2.0), sl, seed=[9, 1, 0])
    cfg = O.OracleConfig(F, normalize=True)
    rho = O.snr_series(noise, bank, cfg, 3 * F, 5 * F)
    filt = O.concatenated_filters(bank, F, O.normalized_mixing(bank))
    ref = O.brute_force(noise, filt, 3 * F, 5 * F)
    np.testing.assert_allclose(rho, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_full_rank_equals_multirate_direct(noise):
    """Full SVD rank reproduces filtering with the uncompressed slices H^s."""
    bank = synth.chirp_bank(F, 8, 20.0, (1.0, 2.0), TINY3, seed=[9, 1, 0], keep_templates=True)
    direct = synth.Bank(bank.n_templates, [synth.Slice(s.rate, s.delay, H, np.eye(H.shape[0]))
                                           for s, H in zip(bank.slices, bank.templates)])
    cfg = O.OracleConfig(F, normalize=False)
    a = O.snr_series(noise, bank, cfg, 2 * F, 4 * F)
    b = O.snr_series(noise, direct, cfg, 2 * F, 4 * F)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-11 * np.abs(b).max())


@pytest.mark.parametrize("sl", [TINY3,
                                [(1024, 0.0, 512, 16), (256, 0.5, 384, 16)],
                                [(1024, 0.0, 128, 16), (128, 0.5, 192, 16)]])
def test_multirate_matches_direct_on_bandlimited_bank(noise, sl):
    """Smooth band-limited templates: the multirate LLOID output equals the
    top-rate direct matched filter to within the resamplers' passband
    accuracy.  Pins the downsampler gain, the slice delays and the
    pre-synchronised look-ahead of every upsampling stage together."""
    bank = synth.burst_bank(F, 8, sl, seed=[9, 1, 0])
    cfg = O.OracleConfig(F, normalize=False)
    rho = O.snr_series(noise, bank, cfg, 3 * F, 5 * F)
    ref = O.brute_force(noise, synth.burst_full_rate(bank, F), 3 * F, 5 * F)
    assert np.abs(rho - ref).max() < 2e-3 * np.abs(ref).max()


def test_self_peak_single_rate_exact():
    """Noiseless strain = A h_cos of template j merging at t0: |z_j| peaks at
    t0 with value A sqrt(1 + <h_s, h_c>^2) (single rate, full rank)."""
    sl = [(1024, 0.0, 2100, 16)]
    bank = synth.chirp_bank(F, 8, 20.0, (1.0, 2.0), sl, seed=[9, 1, 0])
    full = synth.full_rate_templates(bank, F)
    x = np.zeros(6 * F)
    j, t0, A = 3, 3 * F + 517, 12.0
    inj = synth.Injection(0, j, 0, t0, A)
    x2 = x[None].copy()
    synth.inject(x2, F, bank, inj)
    cfg = O.OracleConfig(F, normalize=False)
    z = O.complex_snr(O.snr_series(x2[0], bank, cfg, 3 * F, 4 * F))
    hc, hs = full[2 * j], full[2 * j + 1]
    assert int(np.argmax(np.abs(z[j]))) == t0 - 3 * F
    np.testing.assert_allclose(np.abs(z[j, t0 - 3 * F]), A * np.sqrt(1 + np.dot(hs, hc) ** 2), rtol=1e-10)


def test_self_peak_multirate_full_rank():
    """The plain workload's 2-rate slicing at full rank: the injected
    template's |z| peaks exactly at the merger sample, within 1e-3 of
    A sqrt(1 + <hs,hc>^2).  (At the workload's rank 16 of 128 rows the
    recovered SNR drops to ~0.55 of that and the peak may move one sample.)"""
    w = synth.config1()
    sl = [(r, t, n, 128) for r, t, n, _ in synth.C1_SLICES]
    bank = synth.chirp_bank(2048, 64, 30.0, (2.0, 4.0), sl, seed=[1, 1, 0])
    inj = w.injections[0]
    x = np.zeros((1, w.n_samples))
    synth.inject(x, 2048, bank, inj)
    cfg = O.OracleConfig(2048, normalize=True)
    k = inj.merger_sample // 2048
    z = O.complex_snr(O.snr_series(x[0], bank, cfg, k * 2048, (k + 1) * 2048))
    full = synth.full_rate_templates(bank, 2048)
    hc, hs = full[2 * inj.template], full[2 * inj.template + 1]
    zi = np.abs(z[inj.template])
    assert int(np.argmax(zi)) == inj.merger_sample - k * 2048
    ideal = inj.amplitude * np.sqrt(1 + np.dot(hs, hc) ** 2)
    assert abs(zi.max() / ideal - 1) < 1e-3


def test_noise_invariant_mean_power_is_two():
    """Normalised bank, noise only, after warm-up: mean |z|^2 = 2 (every
    real row has unit norm and the strain unit variance), within 4 standard
    errors from 1-s blocks plus 0.01."""
    w = synth.config1()
    bank = w.banks[0]
    x = synth.gaussian_strain(1, 1, 24 * 2048)[0]
    cfg = O.OracleConfig(2048, normalize=True)
    z, _ = O.lloid_filter(x, bank, cfg, n_strides=16, first_stride=6)
    p = (np.abs(z) ** 2).reshape(z.shape[0], 16, 2048).mean(axis=(0, 2))
    se = p.std(ddof=1) / np.sqrt(len(p))
    assert abs(p.mean() - 2.0) < 4 * se + 0.01


def test_normalisation_is_identity_at_full_rank():
    bank = synth.chirp_bank(F, 8, 20.0, (1.0, 2.0), TINY3, seed=[9, 1, 0])
    n2 = sum((s.mixing ** 2).sum(axis=1) for s in bank.slices)
    assert np.abs(n2 - 1).max() < 2e-2      # sqrt(D) sampling of the slices
    Wn = O.normalized_mixing(bank)
    np.testing.assert_allclose(sum((W ** 2).sum(axis=1) for W in Wn), 1.0, rtol=1e-13)


def test_linearity_and_shift(noise):
    """LLOID is linear in the strain; shifting the strain by a multiple P of
    every rate's decimation factor shifts the output by P."""
    bank = synth.chirp_bank(F, 8, 20.0, (1.0, 2.0), TINY3, seed=[9, 1, 0])
    cfg = O.OracleConfig(F)
    x2 = synth.gaussian_strain(98, 1, 8 * F)[0]
    a = O.snr_series(noise, bank, cfg, 3 * F, 4 * F)
    b = O.snr_series(x2, bank, cfg, 3 * F, 4 * F)
    c = O.snr_series(2.0 * noise - 0.5 * x2, bank, cfg, 3 * F, 4 * F)
    np.testing.assert_allclose(c, 2.0 * a - 0.5 * b, atol=1e-12 * np.abs(c).max())
    P = 4 * 3
    xs = np.concatenate([np.zeros(P), noise])[:len(noise)]
    d = O.snr_series(xs, bank, cfg, 3 * F + P, 4 * F + P)
    np.testing.assert_allclose(d, a, atol=1e-12 * np.abs(a).max())


def test_streaming_equals_batch_for_any_partition(noise):
    bank = synth.chirp_bank(F, 8, 20.0, (1.0, 2.0), TINY3, seed=[9, 1, 0])
    cfg = O.OracleConfig(F)
    x = noise[:5 * F]
    batch = O.complex_snr(O.snr_series(x, bank, cfg, 0, 5 * F))
    for step in (F, F // 2, 3 * F // 4 + 1):
        st = O.LloidStream(bank, cfg)
        parts = [st.push(x[i:i + step]) for i in range(0, len(x), step)]
        np.testing.assert_allclose(np.concatenate(parts, axis=1), batch, rtol=0,
                                   atol=1e-12 * np.abs(batch).max())


def test_streaming_gap_is_zero_strain(noise):
    bank = synth.chirp_bank(F, 8, 20.0, (1.0, 2.0), TINY3, seed=[9, 1, 0])
    cfg = O.OracleConfig(F)
    x = noise[:4 * F].copy()
    s1, s2 = O.LloidStream(bank, cfg), O.LloidStream(bank, cfg)
    out1 = [s1.push(x[k * F:(k + 1) * F], gap=(k == 1)) for k in range(4)]
    x[F:2 * F] = 0
    out2 = [s2.push(x[k * F:(k + 1) * F]) for k in range(4)]
    for a, b in zip(out1, out2):
        np.testing.assert_array_equal(a, b)


def test_latency_condition_is_tight(noise):
    """A slice exactly at the look-ahead limit streams exactly; earlier
    slices are reported.  Two samples earlier the filter reaches strain from
    the future and streaming differs (one sample earlier only the kernel's
    end tap, which the Lanczos window makes exactly zero, would reach it)."""
    chain = [1024, 256]
    la = O.lookahead(chain)
    assert la == [0, 8]
    need = la[1] + O.N_DOWN          # samples at 256 Hz
    for delay, ok in ((need, True), (need - 2, False)):
        sl = [(1024, 0.0, 4 * delay, 8), (256, delay / 256, 200, 8)]
        bank = synth.chirp_bank(F, 4, 40.0, (0.5, 1.2), sl, seed=[9, 1, 0])
        assert (O.latency_violations(bank, F) == []) == ok
        if ok:
            sl1 = [(1024, 0.0, 4 * delay - 4, 8), (256, (delay - 1) / 256, 200, 8)]
            assert O.latency_violations(synth.chirp_bank(F, 4, 40.0, (0.5, 1.2), sl1, seed=[9, 1, 0]), F) == [1]
        cfg = O.OracleConfig(F)
        x = noise[:3 * F]
        batch = O.complex_snr(O.snr_series(x, bank, cfg, 0, 3 * F))
        st = O.LloidStream(bank, cfg)
        strm = np.concatenate([st.push(x[i:i + F]) for i in range(0, 3 * F, F)], axis=1)
        same = np.array_equal(strm, batch) or np.abs(strm - batch).max() < 1e-13
        assert same == ok


def test_lookahead_equals_cumulative_upsampling_half_lengths():
    """Level j look-ahead = sum over the stages from f^s up to the top rate of
    N_up input samples, expressed in level-j samples (pre-synchronisation
    equation of Sec. II.C.3), rounded up to whole samples."""
    for chain in ([4096, 2048, 1024, 512, 256, 128, 64], [4096, 1024, 256], [2048, 512],
                  [4096, 512, 256, 32]):
        la = O.lookahead(chain)
        assert la[0] == 0
        for j in range(1, len(chain)):
            exact = sum(8 * chain[j] / chain[i] for i in range(1, j + 1))
            assert la[j] == int(np.ceil(exact))


def test_window_peaks_first_index_on_ties():
    z = np.array([[1 + 0j, 3j, -3, 2], [0.5, 0.5, 0.5, -0.5j]])
    p = O.window_peaks(z)
    assert list(p.index) == [1, 0]
    np.testing.assert_array_equal(p.snr, [3.0, 0.5])
    assert list(p.above) == [False, False]
    z2 = synth.gaussian_strain(7, 2, 64).view(complex) * 3
    p2 = O.window_peaks(z2)
    np.testing.assert_array_equal(p2.index, np.argmax(np.abs(z2), axis=1))
