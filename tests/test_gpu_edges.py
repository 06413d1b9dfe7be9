"""Degenerate and limit cases of the path (through the C ABI) against the
FP64 oracle: one template / one basis vector / one tap, templates whose
mixing rows are all zero (left unnormalised, output exactly zero), all-zero
strain, the largest basis (160 vectors), the deepest supported decimation
(factor 64, one 64x upsampling stage), a seven-level chain, an odd
detector count, a top rate that is not a power of two (768 Hz), and a clean
rejection beyond the decimation limit."""
import numpy as np
import pytest

import synth
from oracle import lloid as O

from lloid_check import check_peaks, run_gpu, run_oracle, snr_error
from test_gpu_parity import FP32_TOL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F = 4096


@pytest.fixture(scope="module")
def plan_cls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_04730_amd import LloidPlan
    return LloidPlan


def _bank(seed, M, slices):
    """Random bank: per slice (rate, delay, N, L), orthonormal basis rows,
    Gaussian mixing rows decaying with the basis index."""
    g = synth.rng_for(91, synth.PURPOSE_BANK, seed)
    out = []
    for rate, delay, N, L in slices:
        q = np.linalg.qr(g.standard_normal((N, L)))[0]
        W = g.standard_normal((2 * M, L)) * np.exp(-3.0 * np.arange(L) / L)
        out.append(synth.Slice(int(rate), int(delay), np.ascontiguousarray(q.T), np.ascontiguousarray(W)))
    return synth.Bank(M, out)


def _delays(rates, lengths_s, top=F):
    """Delays in slice samples: each slice starts where the previous one
    ends, and no earlier than the look-ahead plus the decimator half-length."""
    la = O.lookahead(sorted(set(rates), reverse=True))
    by_rate = dict(zip(sorted(set(rates), reverse=True), la))
    t, out = 0.0, []
    for r, T in zip(rates, lengths_s):
        need = by_rate[r] + (O.N_DOWN if r < top else 0)
        d = max(int(np.ceil(t * r)), need)
        out.append(d)
        t = (d + T * r) / r
    return out


def _check(plan_cls, banks, n_det, n_strides, seed, precision="fp32", tol=FP32_TOL, top=F):
    x = synth.gaussian_strain(seed, n_det, n_strides * top)
    plan = plan_cls(banks, top, n_det, precision)
    z, pk = run_gpu(plan, x, 0, n_strides)
    for b, bank in enumerate(banks):
        ref = run_oracle(bank, x, top, 0, n_strides)
        eps = snr_error(z[b], ref)
        print(f"bank {b}: eps={eps:.3e}")
        assert eps <= tol
        check_peaks(pk[b], ref, top, float(np.abs(z[b] - ref).max()))
    return z, pk


def test_one_template_one_basis_one_tap(plan_cls):
    b1 = _bank(1, 1, [(4096, 0, 1, 1)])
    d = _delays([4096, 1024], [3 / 4096, 5 / 1024])
    b2 = _bank(2, 1, [(4096, d[0], 3, 1), (1024, d[1], 5, 1)])
    _check(plan_cls, [b1, b2], 1, 3, 201)


def test_zero_mixing_rows_give_zero_output(plan_cls):
    d = _delays([4096, 512], [0.1, 0.5])
    bank = _bank(3, 5, [(4096, d[0], 400, 12), (512, d[1], 256, 9)])
    for s in bank.slices:
        s.mixing[2:4] = 0.0          # template 1: both rows
    z, pk = _check(plan_cls, [bank], 2, 3, 202)
    assert np.all(z[0][:, 1] == 0)
    for p in pk[0]:
        assert np.all(p.snr[:, 1] == 0) and np.all(p.index[:, 1] == 0) and not p.above[:, 1].any()


def test_all_zero_strain(plan_cls):
    d = _delays([4096, 256], [0.05, 1.0])
    bank = _bank(4, 7, [(4096, d[0], 200, 10), (256, d[1], 256, 12)])
    plan = plan_cls([bank], F, 1, "bf16x3")
    z, pk = run_gpu(plan, np.zeros((1, 3 * F)), 0, 3)
    assert np.all(z[0] == 0)
    for p in pk[0]:
        assert np.all(p.snr == 0) and np.all(p.index == 0) and not p.above.any()


def test_largest_basis_and_deepest_decimation(plan_cls):
    """L = 160 basis vectors at the top rate; a 64 Hz slice (decimation 64,
    one upsampling stage of factor 64); three detectors."""
    d = _delays([4096, 64], [200 / 4096, 70 / 64])
    bank = _bank(5, 20, [(4096, d[0], 200, 160), (64, d[1], 70, 50)])
    _check(plan_cls, [bank], 3, 4, 203)
    _check(plan_cls, [bank], 3, 4, 203, precision="bf16x3", tol=1e-4)


def test_seven_level_chain(plan_cls):
    rates = [4096, 2048, 1024, 512, 256, 128, 64]
    lengths = [0.02, 0.05, 0.1, 0.2, 0.4, 0.8, 1.5]
    d = _delays(rates, lengths)
    bank = _bank(6, 9, [(r, dd, max(1, int(T * r)), 6) for r, dd, T in zip(rates, d, lengths)])
    _check(plan_cls, [bank], 1, 4, 204)
    _check(plan_cls, [bank], 1, 4, 204, precision="fp16", tol=1e-3)


def test_top_rate_not_a_power_of_two(plan_cls):
    """Top rate 768 Hz (a multiple of 256, not a power of two): three mixing
    tiles per stride and decimated strides of 384, 96 and 12 samples, the
    last two sharing each output's taps among several threads."""
    top = 768
    rates = [768, 384, 96, 12]
    lengths = [200 / 768, 300 / 384, 150 / 96, 40 / 12]
    d = _delays(rates, lengths, top)
    bank = _bank(8, 11, [(r, dd, max(1, int(round(T * r))), L) for r, dd, T, L in zip(rates, d, lengths, [8, 10, 6, 4])])
    _check(plan_cls, [bank], 2, 6, 205, top=top)
    _check(plan_cls, [bank], 2, 6, 205, precision="bf16x3", tol=1e-4, top=top)


def test_decimation_beyond_the_limit_is_rejected(plan_cls):
    from paper_2511_04730_amd._lib import LloidError
    d = _delays([4096, 32], [0.01, 4.0])
    bank = _bank(7, 4, [(4096, d[0], 40, 4), (32, d[1], 64, 4)])
    with pytest.raises(LloidError) as e:
        plan_cls([bank], F, 1, "fp32")
    assert e.value.status == -7   # LLOID_E_UNSUPPORTED
