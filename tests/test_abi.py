"""C ABI checks that need no GPU: the library loads, exports every function
include/lloid.h declares, and rejects bad arguments on the host before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import lloid as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2511_04730_amd import _lib
    _lib.load()
    return _lib


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lloid.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lloid_[a-z_]+)\s*\(", text)))


def test_every_declared_function_is_exported(L):
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(L):
    lib = L.load()
    for code in range(0, -8, -1):
        assert lib.lloid_status_string(code)
    assert b"look-ahead" in lib.lloid_status_string(-3)


def _create(L, banks, F=1024, n_det=1, precision=0, n_up=8, n_down=32):
    keep = []
    cb = (L.Bank * len(banks))()
    for b, bank in enumerate(banks):
        sl = (L.Slice * len(bank.slices))()
        for i, s in enumerate(bank.slices):
            U = np.ascontiguousarray(s.basis, dtype=np.float64)
            W = np.ascontiguousarray(s.mixing, dtype=np.float64)
            keep += [U, W]
            sl[i] = L.Slice(s.rate, s.delay, U.shape[1], U.shape[0],
                            U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        keep.append(sl)
        cb[b] = L.Bank(bank.n_templates, len(bank.slices), sl)
    cfg = L.Config(F, n_det, n_down, n_up, precision, 1, 4.0)
    h = ctypes.c_void_p()
    return L.load().lloid_plan_create(ctypes.byref(cfg), cb, len(banks), None, ctypes.byref(h))


TINY = [(1024, 0.0, 128, 8), (256, 0.25, 200, 8)]


def test_argument_errors(L):
    lib = L.load()
    h = ctypes.c_void_p()
    assert lib.lloid_plan_create(None, None, 0, None, ctypes.byref(h)) == -1
    bank = synth.chirp_bank(1024, 4, 30.0, (0.5, 1.0), TINY, seed=[1, 1, 0])
    assert _create(L, [bank], n_det=0) == -1
    assert _create(L, [bank], n_up=0) == -1
    assert _create(L, [bank], precision=9) == -1
    assert lib.lloid_plan_query(None, 0, 0, None) == -1
    assert lib.lloid_push_stride(None, None, 0, None, None, None) == -1
    v = ctypes.c_int64()
    assert lib.lloid_plan_query(None, 0, 0, ctypes.byref(v)) == -1


def test_shape_errors(L):
    bank = synth.chirp_bank(1024, 4, 30.0, (0.5, 1.0), TINY, seed=[1, 1, 0])
    assert _create(L, [bank], F=1000) == -2            # top rate not a multiple of the tile
    bad = synth.Bank(4, [synth.Slice(300, 100, bank.slices[0].basis, bank.slices[0].mixing)])
    assert _create(L, [bad]) == -2                      # rate not top / power of two
    big = synth.Bank(4, [synth.Slice(1024, 0, np.zeros((161, 200)), np.zeros((8, 161)))])
    assert _create(L, [big]) == -7                      # more than 160 basis vectors
    deep = synth.Bank(4, [synth.Slice(8, 100, np.zeros((4, 64)), np.zeros((8, 4)))])
    assert _create(L, [deep]) == -7                     # decimation 128 > 64
    neg = synth.Bank(4, [synth.Slice(1024, -1, bank.slices[0].basis, bank.slices[0].mixing)])
    assert _create(L, [neg]) == -2                      # negative delay


def test_latency_error_matches_oracle(L):
    """The library's look-ahead check agrees with the oracle's: at the limit
    the plan is accepted (it then needs a GPU), one sample short it is
    rejected with LLOID_E_LATENCY before any device work."""
    need = O.lookahead([1024, 256])[1] + O.N_DOWN
    short = synth.chirp_bank(1024, 4, 30.0, (0.5, 1.0),
                             [(1024, 0.0, 128, 8), (256, (need - 1) / 256, 200, 8)], seed=[1, 1, 0])
    assert O.latency_violations(short, 1024) == [1]
    assert _create(L, [short]) == -3
    ok = synth.chirp_bank(1024, 4, 30.0, (0.5, 1.0),
                          [(1024, 0.0, 128, 8), (256, need / 256, 200, 8)], seed=[1, 1, 0])
    assert O.latency_violations(ok, 1024) == []
    assert _create(L, [ok]) not in (-1, -2, -3)


def test_noalloc_orthonormalize_host_checks(L):
    """The no-allocation re-orthonormalisation rejects bad sizes on the host
    before any device work: NULL buffers and L < 1 with LLOID_E_ARG, a basis
    larger than its static Gram array (L > 160) with LLOID_E_UNSUPPORTED."""
    lib = L.load()
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: rejected first
    assert lib.lloid_orthonormalize_noalloc(None, 8, 100, fake, 10, None, None) == -1
    assert lib.lloid_orthonormalize_noalloc(fake, 8, 100, None, 10, None, None) == -1
    assert lib.lloid_orthonormalize_noalloc(fake, 0, 100, fake, 10, None, None) == -1
    assert lib.lloid_orthonormalize_noalloc(fake, 8, 7, fake, 10, None, None) == -1
    assert lib.lloid_orthonormalize_noalloc(fake, 161, 400, fake, 10, None, None) == -7


def test_svd_basis_host_checks(L):
    """The SVD construction rejects bad sizes on the host before any device
    work: NULL buffers, L outside 1 .. min(160, rows, N), no iterations, and a
    template matrix of 2^28 doubles or more (its products address it with
    32-bit byte offsets), all with LLOID_E_ARG."""
    lib = L.load()
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: rejected first
    assert lib.lloid_svd_basis(None, 64, 128, 8, 4, fake, fake, None) == -1
    assert lib.lloid_svd_basis(fake, 64, 128, 8, 4, None, fake, None) == -1
    assert lib.lloid_svd_basis(fake, 64, 128, 0, 4, fake, fake, None) == -1
    assert lib.lloid_svd_basis(fake, 64, 128, 65, 4, fake, fake, None) == -1
    assert lib.lloid_svd_basis(fake, 200, 400, 161, 4, fake, fake, None) == -1
    assert lib.lloid_svd_basis(fake, 64, 128, 8, 0, fake, fake, None) == -1
    assert lib.lloid_svd_basis(fake, 1 << 14, 1 << 14, 8, 4, fake, fake, None) == -1
