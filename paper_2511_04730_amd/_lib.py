"""ctypes declarations of the liblloid C ABI (include/lloid.h).

Loading fails loudly when the shared library has not been built: there is
no fallback implementation of any step.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LLOID_LIB may name another build of the same sources (the host-sanitized
# build the tests run the ABI checks against)
LIB_PATH = os.environ.get("LLOID_LIB") or os.path.join(HERE, "liblloid.so")

LLOID_OK = 0
STATUS_NAMES = {0: "LLOID_OK", -1: "LLOID_E_ARG", -2: "LLOID_E_SHAPE", -3: "LLOID_E_LATENCY",
                -4: "LLOID_E_NOMEM", -5: "LLOID_E_HIP", -6: "LLOID_E_STATE", -7: "LLOID_E_UNSUPPORTED"}
PRECISIONS = {"fp32": 0, "bf16x3": 1, "fp16": 2, "fp8_bf16": 3}

Q_N_BANKS, Q_TOTAL_TEMPLATES, Q_SERIES_FLOATS, Q_N_PEAKS = 0, 1, 2, 3
Q_BANK_SERIES_OFFSET, Q_BANK_PEAK_OFFSET, Q_BANK_TEMPLATES, Q_STRIDE = 4, 5, 6, 7
Q_N_SLICES, Q_SLICE_LOOKAHEAD, Q_FLOPS_PER_STRIDE, Q_DEVICE_BYTES = 8, 9, 10, 11
Q_OPTION = 12
OPTIONS = {"graph": 0, "corr_split": 1, "corr_group": 2, "mix_group": 3, "corr_cols": 4, "mix_tblock": 5}
INSPECT_DOWNSAMPLED, INSPECT_BASIS_OUT = 0, 1
KERNEL_NAMES = ["ingest", "down", "corr", "reduce", "mix", "peaks", "xi2", "triggers", "coinc"]


class LloidError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")


class Slice(ctypes.Structure):
    _fields_ = [("rate_hz", ctypes.c_int32), ("delay", ctypes.c_int64), ("n_taps", ctypes.c_int32),
                ("n_basis", ctypes.c_int32), ("basis", ctypes.POINTER(ctypes.c_double)),
                ("mixing", ctypes.POINTER(ctypes.c_double))]


class Bank(ctypes.Structure):
    _fields_ = [("n_templates", ctypes.c_int32), ("n_slices", ctypes.c_int32),
                ("slices", ctypes.POINTER(Slice))]


class Config(ctypes.Structure):
    _fields_ = [("sample_rate_hz", ctypes.c_int32), ("n_detectors", ctypes.c_int32),
                ("n_down", ctypes.c_int32), ("n_up", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("normalize", ctypes.c_int32), ("snr_threshold", ctypes.c_float)]


class WhitenConfig(ctypes.Structure):
    _fields_ = [("n_detectors", ctypes.c_int32), ("block", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("decimation", ctypes.c_int32), ("n_med", ctypes.c_int32), ("n_avg", ctypes.c_int32)]


class Peak(ctypes.Structure):
    _fields_ = [("snr", ctypes.c_float), ("index", ctypes.c_int32), ("re", ctypes.c_float),
                ("im", ctypes.c_float), ("above", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load liblloid.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_04730_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.lloid_plan_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(Bank), ctypes.c_int32, P,
                                      ctypes.POINTER(P)]
    lib.lloid_plan_destroy.argtypes = [P]
    lib.lloid_plan_destroy.restype = None
    lib.lloid_plan_query.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    lib.lloid_push_stride.argtypes = [P, P, ctypes.c_uint32, P, P, P]
    lib.lloid_reset.argtypes = [P, P]
    lib.lloid_state_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.lloid_state_save.argtypes = [P, P, ctypes.c_size_t, P]
    lib.lloid_state_load.argtypes = [P, P, ctypes.c_size_t, P]
    lib.lloid_inspect.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_int64, P, P]
    lib.lloid_profile_enable.argtypes = [P, ctypes.c_int32]
    lib.lloid_profile_read.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
    lib.lloid_grad.argtypes = [P, P, ctypes.c_int32, P, ctypes.POINTER(ctypes.c_double), P, P, P]
    lib.lloid_grad.restype = ctypes.c_int
    lib.lloid_set_slice.argtypes = [P, ctypes.c_int32, P, P, P]
    lib.lloid_set_slice.restype = ctypes.c_int
    lib.lloid_orthonormalize.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P]
    lib.lloid_orthonormalize.restype = ctypes.c_int
    lib.lloid_orthonormalize_noalloc.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P, P]
    lib.lloid_orthonormalize_noalloc.restype = ctypes.c_int
    lib.lloid_set_autocorrelation.argtypes = [P, P, ctypes.POINTER(ctypes.c_int32), P]
    lib.lloid_set_autocorrelation.restype = ctypes.c_int
    lib.lloid_xi2.argtypes = [P, P, P, P, P, P, P]
    lib.lloid_xi2.restype = ctypes.c_int
    lib.lloid_coincidence.argtypes = [P, P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), P, P, P]
    lib.lloid_coincidence.restype = ctypes.c_int
    lib.lloid_whitener_create.argtypes = [ctypes.POINTER(WhitenConfig), P, ctypes.POINTER(P)]
    lib.lloid_whitener_create.restype = ctypes.c_int
    lib.lloid_whitener_destroy.argtypes = [P]
    lib.lloid_whitener_destroy.restype = None
    lib.lloid_whitener_push.argtypes = [P, P, ctypes.c_uint32, P, P]
    lib.lloid_whitener_push.restype = ctypes.c_int
    lib.lloid_whitener_psd.argtypes = [P, P, P]
    lib.lloid_whitener_psd.restype = ctypes.c_int
    lib.lloid_svd_basis.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P]
    lib.lloid_svd_basis.restype = ctypes.c_int
    lib.lloid_quantize_fp8_rows.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P]
    lib.lloid_quantize_fp8_rows.restype = ctypes.c_int
    lib.lloid_set_option.argtypes = [P, ctypes.c_int32, ctypes.c_int64]
    lib.lloid_set_option.restype = ctypes.c_int
    lib.lloid_status_string.argtypes = [ctypes.c_int]
    lib.lloid_status_string.restype = ctypes.c_char_p
    for name in ("lloid_plan_create", "lloid_plan_query", "lloid_push_stride", "lloid_reset",
                 "lloid_state_size", "lloid_state_save", "lloid_state_load", "lloid_inspect",
                 "lloid_profile_enable", "lloid_profile_read"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(status: int, what: str) -> None:
    if status != LLOID_OK:
        raise LloidError(status, what)
