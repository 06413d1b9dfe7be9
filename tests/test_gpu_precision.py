"""Reduced-precision forms against the FP64 oracle.  BF16x3 and FP16 (split
strain and basis outputs) keep the SNR error within 1e-3 (relative above the
trigger threshold, absolute / 4 below); FP8 (e4m3 basis with a power-of-two
scale per basis vector, split e4m3 strain, BF16x3 mixing) has the stated
bound 5e-2, set by the 3-bit mantissa of the basis.  Triggers consistent
within the measured error."""
import numpy as np
import pytest

import synth

from lloid_check import check_peaks, run_gpu, run_oracle, snr_error
from test_gpu_parity import _ragged_banks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EXPECT = {"bf16x3": 1e-4, "fp16": 1e-3, "fp8_bf16": 5e-2}


@pytest.fixture(scope="module")
def plan_cls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_04730_amd import LloidPlan
    return LloidPlan


@pytest.mark.parametrize("precision", ["bf16x3", "fp16", "fp8_bf16"])
def test_ragged_banks_reduced_precision(plan_cls, precision):
    banks = _ragged_banks()
    F = 4096
    x = synth.gaussian_strain(81, 2, 5 * F)
    plan = plan_cls(banks, F, 2, precision)
    z, pk = run_gpu(plan, x, 0, 5)
    for b, bank in enumerate(banks):
        ref = run_oracle(bank, x, F, 0, 5)
        eps = snr_error(z[b], ref)
        print(f"{precision} bank {b} eps={eps:.3e}")
        assert eps <= EXPECT[precision]
        check_peaks(pk[b], ref, F, float(np.abs(z[b] - ref).max()))


@pytest.mark.parametrize("precision", ["bf16x3", "fp16", "fp8_bf16"])
def test_realistic_bank_reduced_precision(plan_cls, precision):
    c2 = synth.cached_workload("c2", synth.config2)
    F = c2.sample_rate
    x = synth.workload_strain(c2, 66)
    plan = plan_cls(c2.banks, F, 1, precision)
    z, pk = run_gpu(plan, x, 65, 1)
    ref = run_oracle(c2.banks[0], x, F, 65, 1)
    eps = snr_error(z[0], ref)
    rms = float(np.sqrt(np.mean(np.abs(z[0] - ref) ** 2) / np.mean(np.abs(ref) ** 2)))
    print(f"realistic bank {precision}: eps={eps:.3e} rel_rms={rms:.3e}")
    assert eps <= EXPECT[precision]
    check_peaks(pk[0], ref, F, float(np.abs(z[0] - ref).max()))


@pytest.mark.parametrize("precision", ["bf16x3", "fp16"])
def test_split_basis_output_rings(plan_cls, precision):
    """The 16-bit forms keep the basis outputs as hi + lo planes of a
    ring grouped by 16 bytes of outputs per position; read back through
    lloid_inspect they match the oracle's correlate step to the form's
    precision."""
    from oracle import lloid as O
    w = synth.config1()
    x = synth.workload_strain(w)
    F = w.sample_rate
    plan = plan_cls(w.banks, F, 1, precision)
    run_gpu(plan, x, 5, 1)
    k, f = 6, 512
    s = w.banks[0].slices[1]
    la = plan.query(9, 1)
    q_lo, q_hi = k * f + la - 400, k * f + la
    y_gpu = plan.basis_out(1, s.n_basis, 0, q_lo, q_hi)
    dd = O.downsample(x[0], 4, q_lo - s.delay - s.n_taps + 1, q_hi - s.delay)
    y_ref = O.correlate(s.basis, dd, q_lo - s.delay - s.n_taps + 1, s.delay, q_lo, q_hi)
    err = np.abs(y_gpu - y_ref).max() / np.abs(y_ref).max()
    print(f"{precision} basis outputs: rel err {err:.3e}")
    assert err < EXPECT[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16", "fp8_bf16"])
def test_set_slice_matches_plan_creation(plan_cls, precision):
    """lloid_set_slice converts a slice exactly as plan creation does in every
    precision form (FP8: e4m3 rows and their per-vector scales), so replacing
    the slices of a plan built for bank A by those of bank B gives the series
    and peaks of a plan built for B, bit for bit."""
    F = 4096
    banks_a = _ragged_banks()
    banks_b = []
    g = np.random.default_rng([7, 5, 1])
    for bank in banks_a:   # same shapes, other values
        sl = [synth.Slice(s.rate, s.delay, g.standard_normal(s.basis.shape) / np.sqrt(s.basis.shape[1]),
                          g.standard_normal(s.mixing.shape) / np.sqrt(s.mixing.shape[1])) for s in bank.slices]
        banks_b.append(synth.Bank(bank.n_templates, sl))
    x = synth.gaussian_strain(85, 2, 3 * F)
    ref = plan_cls(banks_b, F, 2, precision, normalize=False)
    z_ref, p_ref = run_gpu(ref, x, 0, 3)
    plan = plan_cls(banks_a, F, 2, precision, normalize=False)
    k = 0
    for bank in banks_b:
        for s in bank.slices:
            plan.set_slice(k, torch.from_numpy(s.basis).cuda(), torch.from_numpy(s.mixing).cuda())
            k += 1
    z, p = run_gpu(plan, x, 0, 3)
    for b in range(len(banks_b)):
        assert np.array_equal(z[b], z_ref[b]), f"bank {b}"
        for pa, pb in zip(p[b], p_ref[b]):
            assert np.array_equal(pa.index, pb.index) and np.array_equal(pa.snr, pb.snr)


@pytest.mark.parametrize("split", [0, 576])
def test_fp8_basis_outputs_at_fp8_values(plan_cls, split):
    """The FP8 correlation computes exactly the correlation of the FP8 values:
    the basis rows at their e4m3 values with the per-vector scale
    (oracle quantize_fp8_rows) and the decimated stream at its two-part e4m3
    value (hi = e4m3(8 d), lo = e4m3(8 d - hi), saturated at 448), summed
    in FP32 and kept as BF16 hi + lo in the ring: within 2e-4 of the
    oracle's correlate step on those values (the GPU decimates in FP32, which
    can move a sample across an e4m3 rounding boundary).  Slices of 1088 and
    1984 taps (odd multiples of 64: the last 128-tap stage of an item reaches
    past its end) and a 576-tap split (nine 64-tap blocks per item)."""
    from oracle import lloid as O
    F = 2048
    bank = synth.chirp_bank(F, 8, 30.0, (2.0, 4.0), [(2048, 0.0, 1088, 16), (512, 0.5, 1984, 16)],
                            seed=[31, 1, 0])
    x = synth.gaussian_strain(31, 1, 8 * F)
    plan = plan_cls([bank], F, 1, "fp8_bf16", normalize=False)
    if split:
        plan.set_option("corr_split", split)
    run_gpu(plan, x, 7, 1)
    k = 8
    for si, s in enumerate(bank.slices):
        D, f = F // s.rate, s.rate
        la = plan.query(9, si)
        q_lo, q_hi = k * f + la - min(400, f), k * f + la
        y_gpu = plan.basis_out(si, s.n_basis, 0, q_lo, q_hi)
        d_lo = q_lo - s.delay - s.n_taps + 1
        d = O.downsample(x[0], D, d_lo, q_hi - s.delay)
        v = np.clip(d * 8.0, -448.0, 448.0)
        hi = O.e4m3_round(v)
        dq = (hi + O.e4m3_round(v - hi)) / 8.0
        y_ref = O.correlate(O.quantize_fp8_rows(s.basis), dq, d_lo, s.delay, q_lo, q_hi)
        err = np.abs(y_gpu - y_ref).max() / np.abs(y_ref).max()
        print(f"split {split} slice {si} ({s.rate} Hz, {s.n_taps} taps): rel err {err:.3e}", flush=True)
        assert err < 2e-4
