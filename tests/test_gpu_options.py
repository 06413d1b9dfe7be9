"""Tiling options and the autotuner (through the C ABI).

The XCD grouping of work items and the correlation item's column count
change only which work group computes an output, not its summation order,
so results must be bit-identical across them (ragged group counts
included).  The correlation tap split changes the FP32 summation order, so
every split must stay within the FP32 tolerance of the FP64 oracle, also when
it is changed between strides."""
import numpy as np
import pytest

import synth

from lloid_check import check_peaks, run_gpu, run_oracle, snr_error
from test_gpu_parity import FP32_TOL, _ragged_banks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F = 4096


@pytest.fixture(scope="module")
def plan_cls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_04730_amd import LloidPlan
    return LloidPlan


def _peaks_equal(a, b):
    for pa, pb in zip(a, b):
        assert np.array_equal(pa.index, pb.index)
        assert np.array_equal(pa.snr, pb.snr)
        assert np.array_equal(pa.re, pb.re)
        assert np.array_equal(pa.im, pb.im)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_grouping_and_columns_are_bit_exact(plan_cls, precision):
    banks = _ragged_banks()
    x = synth.gaussian_strain(91, 2, 4 * F)
    ref = plan_cls(banks, F, 2, precision)
    ref.set_option("corr_group", 0)
    ref.set_option("mix_group", 0)
    z0, p0 = run_gpu(ref, x, 0, 4)
    for cg, mg, cols, tb in [(16, 32, 256, 1), (3, 5, 64, 3), (64, 256, 192, 16), (1, 1, 128, 64)]:
        plan = plan_cls(banks, F, 2, precision)
        plan.set_option("corr_group", cg)
        plan.set_option("mix_group", mg)
        plan.set_option("corr_cols", cols)
        plan.set_option("mix_tblock", tb)
        assert plan.option("corr_group") == cg and plan.option("mix_group") == mg
        assert plan.option("corr_cols") == cols and plan.option("mix_tblock") == tb
        z, p = run_gpu(plan, x, 0, 4)
        for b in range(len(banks)):
            assert np.array_equal(z[b], z0[b]), f"groups {cg},{mg} bank {b}"
            _peaks_equal(p[b], p0[b])


def test_grouping_change_inside_graph_mode(plan_cls):
    """Changing an option drops the captured graph; the next stride recaptures."""
    banks = _ragged_banks()[:2]
    x = synth.gaussian_strain(92, 2, 4 * F)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    eager = plan_cls(banks, F, 2, "fp32")
    z_ref, _ = run_gpu(eager, x, 0, 4)
    plan = plan_cls(banks, F, 2, "fp32")
    plan.set_graph(True)
    series, peaks = plan.new_series(), plan.new_peaks()
    out = []
    for k in range(4):
        if k == 2:
            plan.set_option("mix_group", 7)
            plan.set_option("corr_group", 0)
            plan.set_option("mix_tblock", 4)
        plan.push(xs[:, k * F:(k + 1) * F].contiguous(), series=series, peaks=peaks)
        out.append([plan.bank_view(series, b).cpu().numpy().astype(np.complex128) for b in range(2)])
    torch.cuda.synchronize()
    for b in range(2):
        assert np.array_equal(np.concatenate([o[b] for o in out], axis=2), z_ref[b])


@pytest.mark.parametrize("split", [64, 192, 65536])
def test_correlation_split_parity(plan_cls, split):
    banks = _ragged_banks()
    x = synth.gaussian_strain(93, 2, 4 * F)
    plan = plan_cls(banks, F, 2, "fp32")
    plan.set_option("corr_split", split)
    assert plan.option("corr_split") == split
    z, pk = run_gpu(plan, x, 0, 4)
    for b, bank in enumerate(banks):
        ref = run_oracle(bank, x, F, 0, 4)
        eps = snr_error(z[b], ref)
        print(f"split {split} bank {b} eps={eps:.3e}")
        assert eps <= FP32_TOL
        check_peaks(pk[b], ref, F, float(np.abs(z[b] - ref).max()))


def test_split_change_between_strides(plan_cls):
    """The split only re-tiles the per-stride work: the stream state carries over."""
    banks = _ragged_banks()
    x = synth.gaussian_strain(94, 2, 5 * F)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    plan = plan_cls(banks, F, 2, "fp32")
    series, peaks = plan.new_series(), plan.new_peaks()
    zs = [[] for _ in banks]
    for k in range(5):
        if k in (2, 4):
            plan.set_option("corr_split", 128 if k == 2 else 4096)
        plan.push(xs[:, k * F:(k + 1) * F].contiguous(), series=series, peaks=peaks)
        for b in range(len(banks)):
            zs[b].append(plan.bank_view(series, b).cpu().numpy().astype(np.complex128))
    torch.cuda.synchronize()
    for b, bank in enumerate(banks):
        ref = run_oracle(bank, x, F, 0, 5)
        assert snr_error(np.concatenate(zs[b], axis=2), ref) <= FP32_TOL


def test_option_values_are_checked(plan_cls):
    from paper_2511_04730_amd._lib import LloidError
    plan = plan_cls(_ragged_banks()[:1], F, 1, "fp32")
    for name, bad in [("corr_split", 0), ("corr_split", 100), ("corr_split", 65600), ("corr_group", -1),
                      ("corr_group", 65), ("mix_group", 257), ("graph", 2), ("corr_cols", 0),
                      ("corr_cols", 100), ("corr_cols", 576), ("mix_tblock", 0), ("mix_tblock", 65)]:
        with pytest.raises(LloidError):
            plan.set_option(name, bad)
    opts = plan.options()
    assert opts["graph"] == 0 and opts["corr_split"] % 64 == 0


def test_autotune_keeps_results(plan_cls):
    from paper_2511_04730_amd.autotune import autotune
    banks = _ragged_banks()
    x = synth.gaussian_strain(95, 2, 4 * F)
    plan = plan_cls(banks, F, 2, "bf16x3")
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    strides = [xs[:, k * F:(k + 1) * F].contiguous() for k in range(3)]
    best = autotune(plan, strides, cols=(64, 256), splits=(256, 1024), corr_groups=(0, 16), mix_groups=(0, 32))
    assert best["corr_split"] in (256, 1024) and best["corr_group"] in (0, 16) and best["mix_group"] in (0, 32)
    assert best["corr_cols"] in (64, 256)
    assert plan.options()["corr_split"] == best["corr_split"]
    assert plan.stride == 0
    z, _ = run_gpu(plan, x, 0, 4)
    for b, bank in enumerate(banks):
        ref = run_oracle(bank, x, F, 0, 4)
        assert snr_error(z[b], ref) <= 1e-4
