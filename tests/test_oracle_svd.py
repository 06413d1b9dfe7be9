"""Pins of the oracle's truncated SVD (Sec. II.C.1), CPU only: full rank
reproduces H; the basis rows are orthonormal; W U = H U^T U; and no other
rank-L projection of the rows (random orthonormal competitors, and the
leading rows of H) leaves a smaller residual (Eckart-Young)."""
import numpy as np

import synth
from oracle import lloid as O


def _H():
    bank = synth.chirp_bank(1024, 10, 25.0, (1.2, 1.5), [(1024, 0.0, 300, 12)], seed=[88, 1, 0],
                            keep_templates=True)
    return np.asarray(bank.templates[0], np.float64)


def test_full_rank_and_orthonormal_rows():
    H = _H()
    U, W = O.svd_truncate(H, H.shape[0])
    assert np.abs(W @ U - H).max() < 1e-12 * np.abs(H).max()
    U, W = O.svd_truncate(H, 7)
    assert np.abs(U @ U.T - np.eye(7)).max() < 1e-13
    assert np.abs(W @ U - H @ U.T @ U).max() < 1e-13 * np.abs(H).max()


def test_truncation_is_the_best_rank_l_projection():
    H = _H()
    L = 6
    U, W = O.svd_truncate(H, L)
    best = np.sum((H - W @ U) ** 2)
    g = synth.rng_for(88, synth.PURPOSE_NOISE, 0)
    for _ in range(50):
        Q = np.linalg.qr(g.standard_normal((H.shape[1], L)))[0].T
        assert np.sum((H - H @ Q.T @ Q) ** 2) >= best
    Q = np.linalg.qr(H[:L].T)[0].T
    assert np.sum((H - H @ Q.T @ Q) ** 2) >= best
