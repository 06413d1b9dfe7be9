"""The no-allocation re-orthonormalisation (lloid_orthonormalize_noalloc),
called through the C ABI, against the allocating entry point
(lloid_orthonormalize) on the same inputs: two calls in a row, the second
with a smaller problem, so that the shared static scratch array is reused
with stale contents from the first call."""
import ctypes

import numpy as np
import pytest

from oracle import lloid as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_04730_amd import _lib
    return _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _case(seed, L, N, rows):
    g = np.random.default_rng([11, seed])
    U = g.standard_normal((L, N)) * np.linspace(1.0, 3.0, L)[:, None]
    W = g.standard_normal((rows, L))
    return U, W


def _run_alloc(L_, U, W):
    Ut, Wt = torch.from_numpy(U.copy()).cuda(), torch.from_numpy(W.copy()).cuda()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L_.check(L_.load().lloid_orthonormalize(_ptr(Ut), U.shape[0], U.shape[1], _ptr(Wt), W.shape[0], st),
             "lloid_orthonormalize")
    return Ut.cpu().numpy(), Wt.cpu().numpy()


def _run_noalloc(L_, U, W, info):
    Ut, Wt = torch.from_numpy(U.copy()).cuda(), torch.from_numpy(W.copy()).cuda()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L_.check(L_.load().lloid_orthonormalize_noalloc(_ptr(Ut), U.shape[0], U.shape[1], _ptr(Wt), W.shape[0],
                                                    _ptr(info) if info is not None else None, st),
             "lloid_orthonormalize_noalloc")
    torch.cuda.synchronize()
    return Ut.cpu().numpy(), Wt.cpu().numpy()


def test_noalloc_matches_allocating_entry_point(lib):
    # first call: L above the in-LDS Cholesky limit (factor in the scratch
    # array itself); second call smaller, in-LDS factor, stale scratch
    info = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    for seed, (L, N, rows) in enumerate([(150, 2000, 300), (24, 500, 64)]):
        U, W = _case(seed, L, N, rows)
        Qa, Wa = _run_alloc(lib, U, W)
        Qn, Wn = _run_noalloc(lib, U, W, info)
        print(f"case L={L} N={N} rows={rows}", flush=True)
        assert info.cpu().tolist() == [0, 0]
        np.testing.assert_array_equal(Qn, Qa)   # same kernels, same order: identical
        np.testing.assert_array_equal(Wn, Wa)
        # and the oracle's CholeskyQR2 to the gradient test's bar
        Qr, Wr = O.cholesky_qr2(U, W)
        np.testing.assert_allclose(Qn @ Qn.T, np.eye(L), atol=1e-12)
        np.testing.assert_allclose(Qn, Qr, atol=1e-10)
        np.testing.assert_allclose(Wn, Wr, atol=1e-10 * np.abs(Wr).max())
        info.fill_(7)


def test_noalloc_reports_breakdown_and_rejects_oversize(lib):
    U, W = _case(5, 16, 300, 20)
    U[3] = 0.0                      # a zero row: the pivot of column 3 is 0
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    _run_noalloc(lib, U, W, info)
    assert info.cpu().tolist()[0] == 4
    Ut, Wt = torch.from_numpy(U.copy()).cuda(), torch.from_numpy(W.copy()).cuda()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.load().lloid_orthonormalize(_ptr(Ut), 16, 300, _ptr(Wt), 20, st) == -6   # LLOID_E_STATE
    # no flag buffer: the flags go to the scratch array, the call still succeeds
    U2, W2 = _case(6, 16, 300, 20)
    Qn, _ = _run_noalloc(lib, U2, W2, None)
    np.testing.assert_allclose(Qn @ Qn.T, np.eye(16), atol=1e-12)
    big = torch.zeros((161, 400), dtype=torch.float64, device="cuda")
    wb = torch.zeros((10, 161), dtype=torch.float64, device="cuda")
    assert lib.load().lloid_orthonormalize_noalloc(_ptr(big), 161, 400, _ptr(wb), 10, None, st) == -7
