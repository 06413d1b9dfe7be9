"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library is rebuilt with every -fsanitize applied to the host pass only
(the device code is unchanged), and two runs load it in a fresh process with
the compiler's shared ASan runtime preloaded and LLOID_LIB pointing at it:
the C-ABI host checks of test_abi.py, and plan creation over several uneven
banks (two detectors, every precision form).  Without a GPU the plan creation
runs argument validation and the host planning that precedes the first
device allocation (rate chains, look-ahead per level, basis-output ring
sizes, series and trigger offsets), then returns LLOID_E_NOMEM; the work
tables, which hold device pointers, are built after it.  Any sanitizer
report fails the run (halt on error).
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _asan_runtime():
    from paper_2511_04730_amd import build
    res = subprocess.run([build.hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True)
    path = res.stdout.strip()
    if res.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    from paper_2511_04730_amd import build
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no shared ASan runtime in this toolchain")
    out = str(tmp_path_factory.mktemp("asan") / "liblloid_asan.so")
    flags = [f for f in build.HIPCC_FLAGS if f != "-O3"] + ["-O1", "-g"]
    host_only = []
    for opt in ("address", "undefined"):
        host_only += ["-Xarch_host", "-fsanitize=" + opt]
    host_only += ["-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-shared-libsan"]
    cmd = [build.hipcc(), *flags, *host_only, "-I", os.path.join(ROOT, "include"),
           *[os.path.join(build.CSRC, s) for s in build.SOURCES], "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]
    env = dict(os.environ, LLOID_LIB=out, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return env


def _clean(res):
    text = res.stdout + res.stderr
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert res.returncode == 0, text[-4000:]


def test_abi_host_checks_under_sanitizers(sanitized):
    res = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q", "-x",
                          "-p", "no:cacheprovider"], capture_output=True, text=True, env=sanitized, cwd=ROOT,
                         timeout=600)
    _clean(res)


PLANNING = r"""
import ctypes, sys
sys.path.insert(0, ROOT); sys.path.insert(0, ROOT + "/tests")
import numpy as np
import synth
from paper_2511_04730_amd import _lib
lib = _lib.load()
assert _lib.LIB_PATH.endswith("liblloid_asan.so")
layouts = [
    [(1024, 0.0, 256, 12), (512, 0.25, 512, 16), (256, 1.0, 768, 20)],
    [(1024, 0.0, 128, 8), (256, 0.5, 400, 24), (128, 2.0, 300, 10), (64, 5.0, 200, 6)],
    [(1024, 0.0, 512, 40), (512, 0.5, 384, 33)],
]
banks = [synth.chirp_bank(1024, 5 + 7 * i, 30.0, (0.5, 3.0), lay, seed=[7, i, 0]) for i, lay in enumerate(layouts)]
keep = []
cb = (_lib.Bank * len(banks))()
for b, bank in enumerate(banks):
    sl = (_lib.Slice * len(bank.slices))()
    for i, s in enumerate(bank.slices):
        U = np.ascontiguousarray(s.basis, dtype=np.float64)
        W = np.ascontiguousarray(s.mixing, dtype=np.float64)
        keep += [U, W]
        sl[i] = _lib.Slice(s.rate, s.delay, U.shape[1], U.shape[0],
                           U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    keep.append(sl)
    cb[b] = _lib.Bank(bank.n_templates, len(bank.slices), sl)
for precision in range(4):
    cfg = _lib.Config(1024, 2, 32, 8, precision, 1, 4.0)
    h = ctypes.c_void_p()
    st = lib.lloid_plan_create(ctypes.byref(cfg), cb, len(banks), None, ctypes.byref(h))
    print("precision", precision, "status", st)
    assert st in (0, -4, -5), st   # with no device: the first allocation fails
    if st == 0:
        lib.lloid_plan_destroy(h)
"""


def test_plan_creation_under_sanitizers(sanitized):
    res = subprocess.run([sys.executable, "-c", f"ROOT = {ROOT!r}\n" + PLANNING], capture_output=True, text=True,
                         env=sanitized, cwd=ROOT, timeout=600)
    _clean(res)
