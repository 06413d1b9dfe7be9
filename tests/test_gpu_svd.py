"""GPU SVD bank construction (Sec. II.C.1) through the C ABI against the
oracle's truncated SVD: the rank-L reconstruction W U (unique when
sigma_L > sigma_{L+1}) element by element, orthonormal basis rows, and the
filter the GPU-built slice gives."""
import numpy as np
import pytest

import synth
from oracle import lloid as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_04730_amd as P
    return P


@pytest.mark.parametrize("L", [4, 12])
def test_svd_basis_matches_oracle(lib, L):
    from paper_2511_04730_amd.plan import svd_basis
    bank = synth.chirp_bank(1024, 10, 25.0, (1.2, 1.5), [(1024, 0.0, 300, 12)], seed=[88, 1, 0],
                            keep_templates=True)
    H = np.asarray(bank.templates[0], np.float64)                 # [20, 300]
    sv = np.linalg.svd(H, compute_uv=False)
    ratio = sv[L] / sv[L - 1]
    iters = int(np.ceil(np.log(1e-14) / (2 * np.log(ratio)))) + 20
    print(f"L={L}: sigma ratio {ratio:.3f}, {iters} iterations")
    g = synth.rng_for(88, synth.PURPOSE_NOISE, 1)
    start = torch.from_numpy(g.standard_normal((L, H.shape[1]))).cuda()
    U, W = svd_basis(torch.from_numpy(H).cuda(), L, start, iters=iters)
    U, W = U.cpu().numpy(), W.cpu().numpy()
    Uo, Wo = O.svd_truncate(H, L)
    err = np.abs(W @ U - Wo @ Uo).max() / np.abs(H).max()
    print(f"reconstruction difference {err:.2e}")
    assert err < 1e-9
    assert np.abs(U @ U.T - np.eye(L)).max() < 1e-12
    assert np.abs(W - H @ U.T).max() < 1e-12 * np.abs(H).max()


def test_rank_deficient_start_is_an_error(lib):
    from paper_2511_04730_amd._lib import LloidError
    from paper_2511_04730_amd.plan import svd_basis
    H = torch.from_numpy(np.random.default_rng(0).standard_normal((8, 64))).cuda()
    with pytest.raises(LloidError) as e:
        svd_basis(H, 3, torch.zeros((3, 64), dtype=torch.float64, device="cuda"), iters=2)
    assert e.value.status == -6
