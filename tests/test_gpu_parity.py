"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import lloid as O

from lloid_check import check_peaks, run_gpu, run_oracle, snr_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP32_TOL = 1e-4      # FP32 products and sums over <= 12k taps: ~1e-6 expected


@pytest.fixture(scope="module")
def plan_cls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_04730_amd import LloidPlan
    return LloidPlan


def _ragged_banks():
    """Three small banks with ragged sizes: M not a multiple of 16, L not a
    multiple of 16, N not a multiple of 64, two slices sharing a rate, a
    bank whose lowest rate is the top rate / 64."""
    F = 4096
    b1 = synth.chirp_bank(F, 21, 30.0, (1.0, 2.5),
                          [(4096, 0.0, 700, 13), (4096, 700 / 4096, 300, 7), (1024, 0.25, 900, 19),
                           (256, 1.25, 333, 22)], seed=[7, 1, 0])
    b2 = synth.chirp_bank(F, 40, 20.0, (2.0, 3.0), [(4096, 0.0, 1024, 33), (512, 0.25, 1400, 40)],
                          seed=[7, 1, 1])
    g = np.random.default_rng([7, 3, 0])
    b3 = synth.random_subbank(g, F, (7, 7), (9, 12), (3.0, 4.0), (20, 40))
    return [b1, b2, b3]


def test_plain_workload_parity(plan_cls):
    """32 s, 2048 Hz, 64 templates, 2 rates: the whole run against the oracle."""
    w = synth.config1()
    x = synth.workload_strain(w)
    plan = plan_cls(w.banks, w.sample_rate, 1, "fp32")
    z, pk = run_gpu(plan, x, 0, 32)
    ref = run_oracle(w.banks[0], x, w.sample_rate, 0, 32)
    eps = snr_error(z[0], ref)
    print(f"plain workload FP32 eps={eps:.3e}")
    assert eps <= FP32_TOL
    e_abs = float(np.abs(z[0] - ref).max())
    check_peaks(pk[0], ref, w.sample_rate, e_abs)
    # the injection is found at its merger sample
    inj = w.injections[0]
    k = inj.merger_sample // w.sample_rate
    assert pk[0][k].snr[0, inj.template] > 4.0


def test_stage_outputs(plan_cls):
    """Decimated stream and basis outputs inside the plan match the oracle's
    downsample and correlate steps."""
    w = synth.config1()
    x = synth.workload_strain(w)
    F = w.sample_rate
    plan = plan_cls(w.banks, F, 1, "fp32")
    run_gpu(plan, x, 5, 1)
    k = 6   # strides pushed
    f = 512
    m_lo, m_hi = k * f - 32 - 600, k * f - 32
    d_gpu = plan.downsampled(4, 0, m_lo, m_hi)
    d_ref = O.downsample(x[0], 4, m_lo, m_hi)
    assert np.abs(d_gpu - d_ref).max() < 1e-5 * np.abs(d_ref).max()
    s = w.banks[0].slices[1]
    la = plan.query(9, 1)
    assert la == O.lookahead([2048, 512])[1]
    q_lo, q_hi = k * f + la - 400, k * f + la
    y_gpu = plan.basis_out(1, s.n_basis, 0, q_lo, q_hi)
    dd = O.downsample(x[0], 4, q_lo - s.delay - s.n_taps + 1, q_hi - s.delay)
    y_ref = O.correlate(s.basis, dd, q_lo - s.delay - s.n_taps + 1, s.delay, q_lo, q_hi)
    assert np.abs(y_gpu - y_ref).max() < 1e-5 * np.abs(y_ref).max()


def test_ragged_multibank_multidetector(plan_cls):
    banks = _ragged_banks()
    F = 4096
    x = synth.gaussian_strain(77, 2, 6 * F)
    plan = plan_cls(banks, F, 2, "fp32")
    z, pk = run_gpu(plan, x, 0, 6)
    for b, bank in enumerate(banks):
        ref = run_oracle(bank, x, F, 0, 6)
        eps = snr_error(z[b], ref)
        print(f"bank {b} eps={eps:.3e}")
        assert eps <= FP32_TOL
        check_peaks(pk[b], ref, F, float(np.abs(z[b] - ref).max()))


def test_gaps_are_zero_strain(plan_cls):
    banks = _ragged_banks()[:2]
    F = 4096
    x = synth.gaussian_strain(78, 2, 4 * F)
    gaps = [0, 0b10, 0b01, 0]
    plan = plan_cls(banks, F, 2, "fp32")
    z, _ = run_gpu(plan, x, 0, 4, gaps=gaps)
    xz = x.copy()
    xz[1, F:2 * F] = 0
    xz[0, 2 * F:3 * F] = 0
    plan2 = plan_cls(banks, F, 2, "fp32")
    z2, _ = run_gpu(plan2, xz, 0, 4)
    for a, b in zip(z, z2):
        assert np.array_equal(a, b)


def test_peaks_only_mode_matches(plan_cls):
    banks = _ragged_banks()
    F = 4096
    x = synth.gaussian_strain(79, 2, 3 * F)
    _, pk1 = run_gpu(plan_cls(banks, F, 2, "fp32"), x, 0, 3)
    _, pk2 = run_gpu(plan_cls(banks, F, 2, "fp32"), x, 0, 3, write_series=False)
    for a, b in zip(pk1, pk2):
        for p, q in zip(a, b):
            assert np.array_equal(p.snr, q.snr) and np.array_equal(p.index, q.index)


def test_deterministic_and_state_resume(plan_cls):
    """Repeat runs are bit-identical; save after k strides, load into a new
    plan, continue: identical to the uninterrupted run."""
    banks = _ragged_banks()
    F = 4096
    x = synth.gaussian_strain(80, 2, 6 * F)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    p1 = plan_cls(banks, F, 2, "fp32")
    p2 = plan_cls(banks, F, 2, "fp32")
    outs1, outs2 = [], []
    for k in range(6):
        s1, _ = p1.push(xs[:, k * F:(k + 1) * F].contiguous())
        outs1.append(s1.cpu())
        if k < 3:
            s2, _ = p2.push(xs[:, k * F:(k + 1) * F].contiguous())
            outs2.append(s2.cpu())
    blob = p2.state_save()
    p3 = plan_cls(banks, F, 2, "fp32")
    p3.state_load(blob)
    assert p3.stride == 3
    for k in range(3, 6):
        s3, _ = p3.push(xs[:, k * F:(k + 1) * F].contiguous())
        outs2.append(s3.cpu())
    for a, b in zip(outs1, outs2):
        assert torch.equal(a, b)
    # reset restarts from zero history
    p1.reset()
    s, _ = p1.push(xs[:, 0:F].contiguous())
    assert torch.equal(s.cpu(), outs1[0])


@pytest.fixture(scope="module")
def c2():
    return synth.cached_workload("c2", synth.config2)


def test_realistic_bank_sampled_parity(plan_cls, c2):
    """The 1024-template, 5-rate bank at full size, in the launch
    configuration the benchmark times: strides 0 (start-up) and 64..65
    (steady state, every slice filled) against the oracle."""
    F = c2.sample_rate
    x = synth.workload_strain(c2, 66)
    plan = plan_cls(c2.banks, F, 1, "fp32")
    z, pk = run_gpu(plan, x, 64, 2)
    ref = run_oracle(c2.banks[0], x, F, 64, 2)
    eps = snr_error(z[0], ref)
    print(f"realistic bank FP32 eps={eps:.3e}")
    assert eps <= FP32_TOL
    check_peaks(pk[0], ref, F, float(np.abs(z[0] - ref).max()))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_graph_replay_matches_direct_launches(plan_cls, precision):
    """One captured HIP graph replayed per stride gives bit-identical series
    and triggers to direct launches, across a gap stride (recapture) and a
    change of output buffer (recapture), with other GPU work and host
    synchronisation between replays."""
    banks = _ragged_banks()
    F = 4096
    x = synth.gaussian_strain(82, 2, 8 * F)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    pe = plan_cls(banks, F, 2, precision)
    pg = plan_cls(banks, F, 2, precision)
    pg.set_graph(True)
    se, sg = pe.new_series(), pg.new_series()
    ke, kg = pe.new_peaks(), pg.new_peaks()
    for k in range(8):
        gap = 0b01 if k == 5 else 0
        if k == 4:
            sg = pg.new_series()
        st = xs[:, k * F:(k + 1) * F].contiguous()
        pe.push(st, gap, series=se, peaks=ke)
        pg.push(st, gap, series=sg, peaks=kg)
        torch.cuda.synchronize()
        assert float((xs * 2.0).sum().item()) != 0.0
        assert torch.equal(se, sg), f"stride {k}"
        assert torch.equal(ke, kg), f"stride {k}"
    assert pg.stride == 8
