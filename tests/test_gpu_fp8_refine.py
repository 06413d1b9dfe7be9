"""Quantisation-aware refinement for the FP8 form (extension) through the C
ABI: the FP8 basis values are bit-exact against the oracle, and refinement
of the mixing rows with every basis held at its FP8 values lowers the loss
monotonically, matches the oracle's loss of the refined bank, and lowers
the FP8 plan's own reconstruction error."""
import numpy as np
import pytest

import synth
from oracle import lloid as O

from test_gpu_grad import F, SL, _target_layout, problem  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_04730_amd as P
    return P


def test_fp8_basis_values_match_oracle(lib):
    from paper_2511_04730_amd.plan import quantize_fp8_rows
    g = synth.rng_for(89, synth.PURPOSE_NOISE, 0)
    U = np.linalg.qr(g.standard_normal((700, 40)))[0].T * g.uniform(1e-3, 30.0, (40, 1))
    U[7] = 0.0
    U[8, :5] = 448.0 * 2.0 ** -20                       # subnormal range after scaling
    got = quantize_fp8_rows(torch.from_numpy(U).cuda()).cpu().numpy()
    assert np.array_equal(got, O.quantize_fp8_rows(U))


def _fp8_loss(lib, bank, x, target, T):
    """Sum over the segment of (rho - target)^2 for a plan in the FP8 form."""
    plan = lib.LloidPlan([bank], F, 1, "fp8_bf16", normalize=False)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    tl = _target_layout(target, bank.n_templates, T).astype(np.float64)
    tot = 0.0
    for k in range(T):
        s, _ = plan.push(xs[:, k * F:(k + 1) * F].contiguous())
        tot += float(np.sum((s.double().cpu().numpy() - tl[k]) ** 2))
    return tot


def test_quantisation_aware_refinement(lib, problem):  # noqa: F811
    from paper_2511_04730_amd.refine import refine
    bank, x, target, T, cfg = problem
    plan = lib.LloidPlan([bank], F, 1, "fp32", normalize=False)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    tg = torch.from_numpy(_target_layout(target, bank.n_templates, T)).cuda()
    losses, U, W = refine(plan, [bank], xs, tg, steps=20, eta=0.12, quantize="fp8")
    print("quantised losses", [f"{v:.4e}" for v in losses[:3]], "...", f"{losses[-1]:.4e}")
    assert losses[-1] < 0.97 * losses[0]
    assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:]))
    for s, u in zip(bank.slices, U):                  # the bases are the FP8 values of the SVD bases
        assert np.array_equal(u.cpu().numpy(), O.quantize_fp8_rows(np.asarray(s.basis)))
    # the oracle's loss of the refined bank
    q_bank = synth.Bank(bank.n_templates, [synth.Slice(s.rate, s.delay, u.cpu().numpy(), w.cpu().numpy())
                                           for s, u, w in zip(bank.slices, U, W)])
    L_ref = O.loss_only(x[0], q_bank, target, cfg, 0, T * F)
    assert abs(losses[-1] - L_ref) <= 1e-4 * L_ref
    # the FP8 plan itself reconstructs the target better with the refined bank
    refined = synth.Bank(bank.n_templates, [synth.Slice(s.rate, s.delay, u.cpu().numpy(), w.cpu().numpy())
                                            for s, u, w in zip(bank.slices, U, W)])
    before, after = _fp8_loss(lib, bank, x, target, T), _fp8_loss(lib, refined, x, target, T)
    print(f"FP8 plan loss: SVD bank {before:.4e}, refined {after:.4e}")
    assert after < before


def test_fp8_refinement_on_the_realistic_bank(lib):
    """The realistic bank (1024 templates, 5 rates, L = 40..120) in the FP8
    form, before and after refining its mixing rows at the FP8 basis values
    (20 steps over the first 72 s of strain, so that every slice, the
    16-64 s one included, sees strain; target = the FP32 output of the
    unrounded bank): the SNR error of the FP8 plan against the FP64 oracle of
    the unrounded bank, at a steady-state stride past the refinement segment,
    drops."""
    from lloid_check import snr_error
    from paper_2511_04730_amd.refine import refine
    c2 = synth.cached_workload("c2", synth.config2)
    bank, Fr = c2.banks[0], c2.sample_rate
    T, k = 72, 80
    x = synth.workload_strain(c2, k + 1)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    seg = xs[:, :T * Fr].contiguous()
    # the refinement filters its segment from zero history; the target is the
    # unrounded bank's FP32 output over the same zero-history segment
    ref = lib.LloidPlan([bank], Fr, 1, "fp32", normalize=False)
    tg = torch.empty((T, ref.series_floats), dtype=torch.float32, device="cuda")
    for i in range(T):
        ref.push(seg[:, i * Fr:(i + 1) * Fr].contiguous(), series=tg[i])
    ref.close()
    plan = lib.LloidPlan([bank], Fr, 1, "fp32", normalize=False)
    losses, U, W = refine(plan, [bank], seg, tg, steps=20, eta=0.25, quantize="fp8")
    print(f"FP8-valued loss {losses[0]:.4e} -> {losses[-1]:.4e}", flush=True)
    assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:])) and losses[-1] < losses[0]
    refined = synth.Bank(bank.n_templates, [synth.Slice(s.rate, s.delay, u.cpu().numpy(), w.cpu().numpy())
                                            for s, u, w in zip(bank.slices, U, W)])
    zr, _ = O.lloid_filter(x[0], bank, O.OracleConfig(Fr, normalize=False), n_strides=1, first_stride=k)
    eps = {}
    for name, b in (("before", bank), ("after", refined)):
        p8 = lib.LloidPlan([b], Fr, 1, "fp8_bf16", normalize=False)
        for i in range(k + 1):
            z, _ = p8.push(xs[:, i * Fr:(i + 1) * Fr].contiguous())
        zg = p8.bank_view(z, 0).cpu().numpy().astype(np.complex128)[0]
        eps[name] = (snr_error(zg, zr), float(np.sqrt(np.mean(np.abs(zg - zr) ** 2) / np.mean(np.abs(zr) ** 2))))
        p8.close()
    print(f"FP8 form vs FP64 oracle of the unrounded bank: eps {eps['before'][0]:.3e} -> {eps['after'][0]:.3e}, "
          f"rel rms {eps['before'][1]:.3e} -> {eps['after'][1]:.3e}", flush=True)
    assert eps["after"][1] < eps["before"][1]
