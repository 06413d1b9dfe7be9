"""Pins of the oracle's loss gradient and re-orthonormalisation (CPU).

The loss is quadratic in every single entry of W^s or U^s (rho is linear in
each), so central finite differences carry no truncation error: only
rounding of order eps * L / h."""
import numpy as np
import pytest

import synth
from oracle import lloid as O

F = 1024
SL = [(1024, 0.0, 96, 6), (512, 0.125, 96, 5), (256, 0.5, 128, 4)]


@pytest.fixture(scope="module")
def setup():
    bank = synth.chirp_bank(F, 4, 25.0, (0.8, 1.0), SL, seed=[11, 1, 0], keep_templates=True)
    cfg = O.OracleConfig(F, normalize=False)
    x = synth.gaussian_strain(11, 1, 4 * F)[0]
    t_lo, t_hi = 2 * F, 2 * F + 300
    target = O.snr_series(x, O.direct_bank(bank), cfg, t_lo, t_hi)
    return bank, cfg, x, target, t_lo, t_hi


@pytest.mark.parametrize("p", [2, 4, 8])
def test_upsample_adjoint_dot_product(p):
    g = np.random.default_rng(p)
    a_lo, a_hi = -20, 60
    i_lo, i_hi = 7 * p - 3, 38 * p + 5
    a = g.standard_normal((3, a_hi - a_lo))
    b = g.standard_normal((3, i_hi - i_lo))
    lhs = np.sum(O.upsample(a, a_lo, p, i_lo, i_hi) * b)
    rhs = np.sum(a * O.upsample_adjoint(b, i_lo, p, a_lo, a_hi))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def _fd(bank, cfg, x, target, t_lo, t_hi, which, s, idx, h=1e-6):
    vals = []
    for sign in (1, -1):
        sl = [synth.Slice(q.rate, q.delay, q.basis.copy(), q.mixing.copy()) for q in bank.slices]
        arr = sl[s].mixing if which == "W" else sl[s].basis
        arr[idx] += sign * h
        vals.append(O.loss_only(x, synth.Bank(bank.n_templates, sl), target, cfg, t_lo, t_hi))
    return (vals[0] - vals[1]) / (2 * h)


def test_gradient_matches_central_differences(setup):
    bank, cfg, x, target, t_lo, t_hi = setup
    L, dW, dU = O.loss_and_grad(x, bank, target, cfg, t_lo, t_hi)
    assert L > 0
    g = np.random.default_rng(5)
    for s, sl in enumerate(bank.slices):
        for _ in range(3):
            idx = (int(g.integers(sl.mixing.shape[0])), int(g.integers(sl.mixing.shape[1])))
            fd = _fd(bank, cfg, x, target, t_lo, t_hi, "W", s, idx)
            assert abs(fd - dW[s][idx]) <= 1e-6 * max(1.0, np.abs(dW[s]).max()), ("W", s, idx, fd, dW[s][idx])
            idx = (int(g.integers(sl.basis.shape[0])), int(g.integers(sl.basis.shape[1])))
            fd = _fd(bank, cfg, x, target, t_lo, t_hi, "U", s, idx)
            assert abs(fd - dU[s][idx]) <= 1e-6 * max(1.0, np.abs(dU[s]).max()), ("U", s, idx, fd, dU[s][idx])


def test_gradient_vanishes_at_full_rank(setup):
    """With every slice at full rank the compressed filter equals the
    direct one, the residual and hence the gradient vanish."""
    _, cfg, x, _, t_lo, t_hi = setup
    full = synth.chirp_bank(F, 4, 25.0, (0.8, 1.0), [(r, t, n, 8) for r, t, n, _ in SL], seed=[11, 1, 0],
                            keep_templates=True)
    target = O.snr_series(x, O.direct_bank(full), cfg, t_lo, t_hi)
    L, dW, dU = O.loss_and_grad(x, full, target, cfg, t_lo, t_hi)
    scale = np.sum(target ** 2)
    assert L < 1e-20 * scale
    assert max(np.abs(d).max() for d in dW + dU) < 1e-8


def test_cholesky_qr2_orthonormal_and_invariant():
    g = np.random.default_rng(3)
    U = g.standard_normal((7, 300)) * np.linspace(1, 5, 7)[:, None]
    W = g.standard_normal((10, 7))
    Q, W2 = O.cholesky_qr2(U, W)
    np.testing.assert_allclose(Q @ Q.T, np.eye(7), atol=1e-13)
    np.testing.assert_allclose(W2 @ Q, W @ U, atol=1e-12 * np.abs(W @ U).max())
    # the rows span the same space: Q is U's row space (compare with numpy QR)
    Qn, _ = np.linalg.qr(U.T)
    np.testing.assert_allclose(np.abs(Qn.T @ Q.T), np.eye(7), atol=1e-12)


def test_planted_gradient_slip_is_caught(setup, monkeypatch):
    """A one-sample slip in the transposed upsampler breaks the FD pin."""
    bank, cfg, x, target, t_lo, t_hi = setup
    orig = O.upsample_adjoint

    def slipped(g, g_lo, p, a_lo, a_hi, n_up=O.N_UP):
        out = orig(g, g_lo, p, a_lo, a_hi, n_up)
        return np.concatenate([out[:, 1:], np.zeros((out.shape[0], 1))], axis=1)

    monkeypatch.setattr(O, "upsample_adjoint", slipped)
    L, dW, dU = O.loss_and_grad(x, bank, target, cfg, t_lo, t_hi)
    s = 2
    idx = (1, 5)
    fd = _fd(bank, cfg, x, target, t_lo, t_hi, "U", s, idx)
    assert abs(fd - dU[s][idx]) > 1e-4 * max(1.0, np.abs(dU[s]).max())
