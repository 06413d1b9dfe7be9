"""Parity of the batched workloads against the FP64 oracle, through the C ABI.

Batched (200 uneven sub-banks, 120333 templates, 3-7 rates down to 64 Hz,
filters up to 64 s, 2 detectors; the headline): the triggers of every
template and detector at stride 64 (steady state) against the oracle's,
stored by tests/golden/make_batched_triggers.py, and the full SNR series of
that stride for 40 banks (every rate count from 3 to 7 and the bank with the
longest slice) against the oracle computed here, in BF16x3 and FP32.

Largest (20 sub-banks of the 800-bank workload: the 10 six-rate banks with
the longest filters, down to 128 Hz and up to 127 s, and the 10 other banks
with the longest slices, up to 97k taps; 2 detectors): series and triggers
at stride 128 (steady state) in the FP8 form (stated bound 5e-2) and FP32.
"""
import os

import numpy as np
import pytest

import synth
from oracle import lloid as O
from lloid_check import check_peaks, oracle_series, snr_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batched_triggers_stride64.npz")
K3 = 64
K5 = 128


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_04730_amd as P
    return P


def run_to_stride(plan, x, F, k):
    """Push strides 0..k (series written only at stride k); returns the
    series and peaks tensors of stride k."""
    xs = torch.from_numpy(np.ascontiguousarray(x[:, :(k + 1) * F].astype(np.float32))).cuda()
    series = plan.new_series()
    peaks = plan.new_peaks()
    for i in range(k + 1):
        plan.push(xs[:, i * F:(i + 1) * F].contiguous(), series=series, peaks=peaks, write_series=(i == k))
    torch.cuda.synchronize()
    return series, peaks


def check_golden_triggers(plan, peaks, golden, tol):
    """Every GPU trigger against the stored oracle triggers: the index must be
    a stored near-maximum sample within 2 e_abs of the oracle maximum p
    (e_abs = tol max(p, 4)), the oracle's own index when no other sample is
    that close; |z| within 2 e_abs of p, z within 4 e_abs of the oracle's
    value at that index, the threshold flag equal away from the threshold."""
    g_idx, g_snr, g_re, g_im, g_above = [], [], [], [], []
    for b in range(plan.n_banks):
        pv = plan.peaks_view(peaks, b)
        g_idx.append(pv.index.reshape(-1))
        g_snr.append(pv.snr.reshape(-1))
        g_re.append(pv.re.reshape(-1))
        g_im.append(pv.im.reshape(-1))
        g_above.append(pv.above.reshape(-1))
    g_idx, g_snr, g_re, g_im, g_above = map(np.concatenate, (g_idx, g_snr, g_re, g_im, g_above))
    count = golden["count"]
    assert len(count) == len(g_idx)
    off = np.concatenate([[0], np.cumsum(count)[:-1]])
    cz = golden["re"].astype(np.float64) + 1j * golden["im"].astype(np.float64)
    p = np.abs(cz[off])
    e_abs = tol * np.maximum(p, 4.0)
    assert np.all(2 * e_abs < golden["tau"] * np.maximum(p, 4.0))   # the stored set covers every allowed index
    tid = np.repeat(np.arange(len(count)), count)
    allowed = np.abs(cz) >= (p - 2 * e_abs)[tid]
    allowed[off] = True
    hit = allowed & (golden["index"] == g_idx[tid])
    n_hit = np.bincount(tid, weights=hit, minlength=len(count))
    bad = np.nonzero(n_hit == 0)[0]
    assert len(bad) == 0, f"{len(bad)} trigger indices outside the oracle's near-maximum set, first {bad[:5]}"
    zsel = np.zeros(len(count), complex)
    zsel[tid[hit]] = cz[hit]
    assert np.all(np.abs(g_snr - p) <= 2 * e_abs), np.max(np.abs(g_snr - p) / e_abs)
    dz = np.abs((g_re + 1j * g_im) - zsel)
    assert np.all(dz <= 4 * e_abs), np.max(dz / e_abs)
    clear = np.abs(p - 4.0) > 2 * e_abs
    assert np.array_equal(g_above[clear].astype(bool), (p >= 4.0)[clear])
    exact = np.bincount(tid, weights=allowed, minlength=len(count)) == 1
    return int(exact.sum()), len(count)


def _series_banks(w):
    """40 banks: per rate count 3..7 the first seven banks with it, the bank
    with the longest slice, and the first banks not yet taken."""
    R = [len(b.slices) for b in w.banks]
    pick = []
    for r in range(3, 8):
        pick += [i for i in range(len(w.banks)) if R[i] == r][:7]
    longest = int(np.argmax([max(s.n_taps for s in b.slices) for b in w.banks]))
    if longest not in pick:
        pick.append(longest)
    for i in range(len(w.banks)):
        if len(pick) >= 40:
            break
        if i not in pick:
            pick.append(i)
    return sorted(pick), longest


@pytest.fixture(scope="module")
def batched():
    w = synth.cached_workload("c3", synth.config3)
    x = synth.workload_strain(w, K3 + 1)
    golden = dict(np.load(GOLDEN, allow_pickle=False))
    import importlib.util
    spec = importlib.util.spec_from_file_location("mk", os.path.join(os.path.dirname(GOLDEN), "make_batched_triggers.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    assert int(golden["stride"]) == K3
    np.testing.assert_allclose(golden["fingerprint"], mk.fingerprint(w, x), rtol=1e-12)
    pick, longest = _series_banks(w)
    print(f"oracle series of {len(pick)} banks at stride {K3} ...", flush=True)
    zref = oracle_series([w.banks[b] for b in pick], x, w.sample_rate, K3)
    return w, x, golden, pick, longest, zref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision, tol", [("bf16x3", 1e-4), ("fp32", 1e-5)])
def test_batched_workload_all_banks(lib, batched, precision, tol):
    w, x, golden, pick, longest, zref = batched
    F = w.sample_rate
    plan = lib.LloidPlan(w.banks, F, w.n_detectors, precision)
    series, peaks = run_to_stride(plan, x, F, K3)
    n_exact, n = check_golden_triggers(plan, peaks, golden, tol)
    print(f"{precision}: {n} triggers (2 det x {w.n_templates} templates) match the oracle, "
          f"{n_exact} with a unique near-maximum", flush=True)
    eps = 0.0
    rates = set()
    for b, z in zip(pick, zref):
        zg = plan.bank_view(series, b).cpu().numpy().astype(np.complex128)
        e = snr_error(zg, z)
        eps = max(eps, e)
        rates.add(len(w.banks[b].slices))
        assert e <= tol, f"bank {b}: {e}"
        e_abs = float(np.abs(zg - z).max())
        pv = plan.peaks_view(peaks, b)
        check_peaks([pv], z, F, max(e_abs, 1e-7))
    assert rates == {3, 4, 5, 6, 7} and longest in pick
    print(f"{precision}: series of {len(pick)} banks (rates 3..7, longest slice "
          f"{max(s.n_taps for s in w.banks[longest].slices)} taps) eps = {eps:.3e}", flush=True)
    plan.close()


@pytest.fixture(scope="module")
def largest():
    shapes = synth.config5_shapes()
    six = [i for i, sh in enumerate(shapes) if sh[1] == 6]
    longest_t = sorted(six, key=lambda i: -shapes[i][2])[:10]          # 128 Hz, filters up to 128 s
    longest_n = [i for i in sorted(range(len(shapes)), key=lambda i: -shapes[i][3]) if i not in longest_t][:10]
    idx = sorted(longest_t + longest_n)                                 # ... and the longest slices (97k taps)
    banks = synth.config5_banks(idx)
    x = synth.gaussian_strain(5, 2, (K5 + 1) * 4096)
    print(f"oracle series of {len(banks)} banks at stride {K5} ...", flush=True)
    zref = oracle_series(banks, x, 4096, K5)
    return idx, banks, x, zref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision, tol", [("fp8_bf16", 5e-2), ("fp32", 1e-5)])
def test_largest_workload_longest_banks(lib, largest, precision, tol):
    idx, banks, x, zref = largest
    F = 4096
    plan = lib.LloidPlan(banks, F, 2, precision)
    series, peaks = run_to_stride(plan, x, F, K5)
    eps = 0.0
    for b, z in enumerate(zref):
        zg = plan.bank_view(series, b).cpu().numpy().astype(np.complex128)
        e = snr_error(zg, z)
        eps = max(eps, e)
        assert e <= tol, f"bank {idx[b]}: {e}"
        check_peaks([plan.peaks_view(peaks, b)], z, F, max(float(np.abs(zg - z).max()), 1e-7))
    nmax = max(s.n_taps for b in banks for s in b.slices)
    assert nmax > 90000 and min(s.rate for b in banks for s in b.slices) == 128
    print(f"{precision}: {len(banks)} banks ({sum(b.n_templates for b in banks)} templates, longest slice "
          f"{nmax} taps, rates down to 128 Hz), 2 det, stride {K5}: eps = {eps:.3e}", flush=True)
    plan.close()
