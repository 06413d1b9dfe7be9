"""The gradient and refinement at the gradient workload's shape: the
realistic bank (1024 templates, 5 rates 4096..256 Hz, slices of 1024 to
12288 taps) truncated to half its basis counts (L = 20/30/40/50/60), 4096 Hz.

1. Backward arithmetic against the FP64 oracle on 64 of the templates over
   20 s (the 16-64 s slice sees strain in the last 4 s), with a known
   residual E (target = the plan's own output - E, the oracle's target its
   own output - E): every slice's dW and dU, including the split-K paths
   (20 x 4096 time samples: 107 dW splits and ten dU splits at the top
   rate).
2. 100 refinement steps on the whole bank over 64 s with FP64 CholeskyQR2
   on the GPU after each: loss non-increasing, orthonormal bases to 1e-12,
   W U unchanged by a re-orthonormalisation, and the refined bank's series
   at one stride equal to the oracle's for the same refined bank.  The
   target is the FP32 output of the same bank at its full basis counts
   (L = 40/60/80/100/120; the multirate-direct target at this size is too
   slow for the oracle here).
"""
import numpy as np
import pytest

import synth
from oracle import lloid as O
from lloid_check import snr_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F = 4096


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_04730_amd as P
    return P


@pytest.fixture(scope="module")
def full_bank():
    return synth.config2(duration_s=64).banks[0]


def _series(plan, xs, T):
    plan.reset()
    out = []
    for k in range(T):
        s, _ = plan.push(xs[:, k * F:(k + 1) * F].contiguous())
        out.append(s.clone())
    torch.cuda.synchronize()
    return torch.stack(out)


def _rows_layout(E, M, T):
    z = E[0::2] + 1j * E[1::2]
    z = z.reshape(M, T, F).transpose(1, 0, 2)
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1).reshape(T, M * F * 2))


@pytest.mark.timeout(600)
def test_backward_at_gradient_workload_shape(lib, full_bank):
    half = synth.truncate_bank(full_bank, synth.C4_BASIS)
    rows = np.arange(0, 1024, 16)
    r2 = np.sort(np.concatenate([2 * rows, 2 * rows + 1]))
    bank = synth.Bank(len(rows), [synth.Slice(s.rate, s.delay, s.basis, np.ascontiguousarray(s.mixing[r2]))
                                  for s in half.slices])
    T = 20
    x = synth.gaussian_strain(4, 1, T * F)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    plan = lib.LloidPlan([bank], F, 1, "fp32", normalize=False)
    E = np.random.default_rng([4, 9]).standard_normal((2 * bank.n_templates, T * F)) * 0.1
    tg = _series(plan, xs, T).double().cpu().numpy() - _rows_layout(E, bank.n_templates, T)
    loss, dW, dU = plan.grad(xs, torch.from_numpy(tg.astype(np.float32)).cuda())
    cfg = O.OracleConfig(F, normalize=False)
    rho = O.snr_series(x[0], bank, cfg, 0, T * F, mixing=[s.mixing for s in bank.slices])
    L_ref, dW_ref, dU_ref = O.loss_and_grad(x[0], bank, rho - E, cfg, 0, T * F)
    print(f"loss gpu {loss:.6e} oracle {L_ref:.6e}", flush=True)
    assert abs(loss - L_ref) <= 1e-5 * L_ref
    for s in range(len(bank.slices)):
        ew = np.abs(dW[s].cpu().numpy() - dW_ref[s]).max() / np.abs(dW_ref[s]).max()
        eu = np.abs(dU[s].cpu().numpy() - dU_ref[s]).max() / np.abs(dU_ref[s]).max()
        sl = bank.slices[s]
        print(f"slice {s} ({sl.rate} Hz, N {sl.n_taps}, L {sl.n_basis}): dW rel err {ew:.2e}, dU rel err {eu:.2e}",
              flush=True)
        assert ew < 1e-4 and eu < 1e-4
    # the 16-64 s slice: only its latest 4 s of taps see the 20 s of strain
    last = np.abs(dU_ref[4]).max(axis=0) > 0
    assert last[-4 * 256:].all() and not last[:-4 * 256 - 128].any()


@pytest.mark.timeout(900)
def test_refinement_on_the_whole_gradient_workload(lib, full_bank):
    from paper_2511_04730_amd.plan import orthonormalize
    from paper_2511_04730_amd.refine import refine
    half = synth.truncate_bank(full_bank, synth.C4_BASIS)
    T = 64
    x = synth.gaussian_strain(4, 1, T * F)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    target_plan = lib.LloidPlan([full_bank], F, 1, "fp32", normalize=False)
    tg = _series(target_plan, xs, T)
    target_plan.close()
    plan = lib.LloidPlan([half], F, 1, "fp32", normalize=False)
    # steps: mixing rows eta = 0.25, bases 0.1 / sigma_max^2 (the loss rose
    # within five steps with 0.5 / sigma_max^2 for the bases)
    smax2 = max(float(np.linalg.norm(s.mixing, 2)) ** 2 for s in half.slices)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    losses, U, W = refine(plan, [half], xs, tg, steps=100, eta=0.25, eta_u=0.1 / smax2)
    ev1.record()
    torch.cuda.synchronize()
    print(f"100 steps in {ev0.elapsed_time(ev1) / 1e3:.2f} s; loss {losses[0]:.6e} -> {losses[-1]:.6e} "
          f"(sigma_max^2 {smax2:.1f})", flush=True)
    assert all(b <= a * (1 + 1e-7) for a, b in zip(losses, losses[1:])), losses
    assert losses[-1] < losses[0]
    for u in U:
        un = u.cpu().numpy()
        np.testing.assert_allclose(un @ un.T, np.eye(un.shape[0]), atol=1e-12)
    # W U unchanged by one more re-orthonormalisation
    for u, wt in zip(U, W):
        u2, w2 = u.clone(), wt.clone()
        orthonormalize(u2, w2)
        before = (wt @ u).cpu().numpy()
        after = (w2 @ u2).cpu().numpy()
        np.testing.assert_allclose(after, before, atol=1e-12 * np.abs(before).max())
    # the refined bank filters as the oracle says, at a steady-state stride
    refined = synth.Bank(half.n_templates, [synth.Slice(s.rate, s.delay, u.cpu().numpy(), wt.cpu().numpy())
                                            for s, u, wt in zip(half.slices, U, W)])
    k = T - 1
    plan.reset()
    for i in range(k + 1):
        z, _ = plan.push(xs[:, i * F:(i + 1) * F].contiguous())
    zg = plan.bank_view(z, 0).cpu().numpy().astype(np.complex128)
    zr, _ = O.lloid_filter(x[0, :(k + 1) * F], refined, O.OracleConfig(F, normalize=False), n_strides=1,
                           first_stride=k)
    eps = snr_error(zg[0], zr)
    print(f"refined bank, stride {k}: eps = {eps:.3e}", flush=True)
    assert eps <= 1e-5
