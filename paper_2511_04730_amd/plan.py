"""Python face of the LLOID C ABI: argument marshalling only.

Every step of the filtering runs in liblloid's HIP kernels; torch provides
device memory (tensors) and the HIP stream the work is enqueued on.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L


@dataclass
class PeakArrays:
    snr: "np.ndarray"
    index: "np.ndarray"
    re: "np.ndarray"
    im: "np.ndarray"
    above: "np.ndarray"


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class LloidPlan:
    """One plan = a set of banks filtered together, for n_detectors streams.

    banks: sequence of objects with ``n_templates`` and ``slices``; each
    slice has ``rate``, ``delay``, ``basis`` [L, N] and ``mixing`` [2M, L]
    (float64 arrays)."""

    def __init__(self, banks: Sequence, sample_rate: int, n_detectors: int = 1, precision: str = "fp32",
                 normalize: bool = True, n_down: int = 32, n_up: int = 8, snr_threshold: float = 4.0,
                 stream=None):
        import torch
        self.lib = L.load()
        self.sample_rate = int(sample_rate)
        self.n_detectors = int(n_detectors)
        self.precision = precision
        keep = []
        cbanks = (L.Bank * len(banks))()
        for b, bank in enumerate(banks):
            sl = (L.Slice * len(bank.slices))()
            for i, s in enumerate(bank.slices):
                U = np.ascontiguousarray(s.basis, dtype=np.float64)
                W = np.ascontiguousarray(s.mixing, dtype=np.float64)
                keep += [U, W]
                sl[i] = L.Slice(int(s.rate), int(s.delay), U.shape[1], U.shape[0],
                                U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
            keep.append(sl)
            cbanks[b] = L.Bank(int(bank.n_templates), len(bank.slices), sl)
        cfg = L.Config(self.sample_rate, self.n_detectors, n_down, n_up, L.PRECISIONS[precision],
                       1 if normalize else 0, float(snr_threshold))
        handle = ctypes.c_void_p()
        st = _stream_handle(stream) if torch.cuda.is_available() else None
        L.check(self.lib.lloid_plan_create(ctypes.byref(cfg), cbanks, len(banks), st, ctypes.byref(handle)),
                "lloid_plan_create")
        self.handle = handle
        self._banks_meta = [[(int(np.shape(s.basis)[0]), int(np.shape(s.basis)[1])) for s in bank.slices]
                            for bank in banks]
        self.n_banks = self.query(L.Q_N_BANKS)
        self.series_floats = self.query(L.Q_SERIES_FLOATS)
        self.n_peaks = self.query(L.Q_N_PEAKS)
        self.bank_templates = [self.query(L.Q_BANK_TEMPLATES, b) for b in range(self.n_banks)]
        self.bank_series_offset = [self.query(L.Q_BANK_SERIES_OFFSET, b) for b in range(self.n_banks)]
        self.bank_peak_offset = [self.query(L.Q_BANK_PEAK_OFFSET, b) for b in range(self.n_banks)]
        self.flops_per_stride = self.query(L.Q_FLOPS_PER_STRIDE)

    def set_graph(self, enable: bool = True) -> None:
        """Replay one captured HIP graph per stride (LLOID_OPT_GRAPH)."""
        self.set_option("graph", 1 if enable else 0)

    def set_option(self, name: str, value: int) -> None:
        """lloid_set_option by name: graph, corr_split, corr_cols, corr_group, mix_group, mix_tblock."""
        L.check(self.lib.lloid_set_option(self.handle, L.OPTIONS[name], int(value)), "lloid_set_option")

    def option(self, name: str) -> int:
        return self.query(L.Q_OPTION, L.OPTIONS[name])

    def options(self) -> dict:
        return {k: self.option(k) for k in L.OPTIONS}

    def query(self, what: int, index: int = 0) -> int:
        v = ctypes.c_int64()
        L.check(self.lib.lloid_plan_query(self.handle, what, index, ctypes.byref(v)), "lloid_plan_query")
        return int(v.value)

    @property
    def stride(self) -> int:
        return self.query(L.Q_STRIDE)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.lloid_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ outputs
    def new_series(self):
        import torch
        return torch.empty(self.series_floats, dtype=torch.float32, device="cuda")

    def new_peaks(self):
        import torch
        return torch.empty(self.n_peaks * 5, dtype=torch.int32, device="cuda")

    def push(self, strain, gap_mask: int = 0, series=None, peaks=None, write_series: bool = True, stream=None):
        """Filter the next stride.  strain: cuda float32 [n_det, F].
        Returns (series or None, peaks) device tensors (see bank_view /
        peaks_view for per-bank shapes)."""
        import torch
        assert strain.is_cuda and strain.dtype == torch.float32 and strain.is_contiguous()
        assert tuple(strain.shape) == (self.n_detectors, self.sample_rate)
        if write_series and series is None:
            series = self.new_series()
        if peaks is None:
            peaks = self.new_peaks()
        sptr = ctypes.c_void_p(series.data_ptr()) if write_series else None
        L.check(self.lib.lloid_push_stride(self.handle, ctypes.c_void_p(strain.data_ptr()), int(gap_mask), sptr,
                                           ctypes.c_void_p(peaks.data_ptr()), _stream_handle(stream)),
                "lloid_push_stride")
        return (series if write_series else None), peaks

    def bank_view(self, series, bank: int):
        """[n_det, M_b, F] complex64 view of one bank's block of a series tensor."""
        import torch
        M = self.bank_templates[bank]
        off = self.bank_series_offset[bank]
        blk = series[off:off + self.n_detectors * M * self.sample_rate * 2]
        return torch.view_as_complex(blk.view(self.n_detectors, M, self.sample_rate, 2))

    def peaks_view(self, peaks, bank: int) -> PeakArrays:
        """Host arrays [n_det, M_b] of one bank's triggers."""
        M = self.bank_templates[bank]
        off = self.bank_peak_offset[bank]
        raw = peaks.view(-1, 5)[off:off + self.n_detectors * M].cpu().numpy()
        f = raw.view(np.float32)
        shp = (self.n_detectors, M)
        return PeakArrays(f[:, 0].reshape(shp).copy(), raw[:, 1].reshape(shp).copy(), f[:, 2].reshape(shp).copy(),
                          f[:, 3].reshape(shp).copy(), raw[:, 4].reshape(shp).copy())

    # ------------------------------------------------------------ xi^2
    def set_autocorrelation(self, acf, lengths, stream=None) -> None:
        """Store the template autocorrelations for xi2(): acf is a cuda
        float64 tensor holding, bank after bank, [M_b, A_b, 2] blocks of
        (re, im) R(t), t = -(A_b-1)/2 .. (A_b-1)/2; lengths = [A_b]."""
        import torch
        assert acf.is_cuda and acf.dtype == torch.float64 and acf.is_contiguous()
        A = (ctypes.c_int32 * self.n_banks)(*[int(a) for a in lengths])
        assert acf.numel() == sum(2 * M * a for M, a in zip(self.bank_templates, lengths))
        L.check(self.lib.lloid_set_autocorrelation(self.handle, ctypes.c_void_p(acf.data_ptr()), A,
                                                   _stream_handle(stream)), "lloid_set_autocorrelation")

    def xi2(self, cur, peaks, prev=None, next=None, out=None, stream=None):
        """xi^2 at the triggers `peaks` of the stride whose series is `cur`
        (prev / next: the neighbouring strides' series, or None).  Returns a
        cuda float32 tensor [n_peaks], in the order of the triggers."""
        import torch
        if out is None:
            out = torch.empty(self.n_peaks, dtype=torch.float32, device="cuda")
        ptr = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None)
        L.check(self.lib.lloid_xi2(self.handle, ptr(prev), ptr(cur), ptr(next), ptr(peaks), ptr(out),
                                   _stream_handle(stream)), "lloid_xi2")
        return out

    def xi2_view(self, xi2, bank: int) -> "np.ndarray":
        """Host array [n_det, M_b] of one bank's xi^2 values."""
        M = self.bank_templates[bank]
        off = self.bank_peak_offset[bank]
        return xi2[off:off + self.n_detectors * M].cpu().numpy().reshape(self.n_detectors, M)

    # ------------------------------------------------------------ coincidence
    def coincidence(self, peaks, window, overlap: int, prev=None, triggers=None, events=None, stream=None):
        """Window triggers (last `overlap` samples of the previous stride's
        series `prev` plus this stride's `peaks`), coincident events and one
        event per bank.  window: [n_det][n_det] samples.  Returns (triggers,
        events): device tensors in the peaks layout and [n_banks, 4] int32
        (network SNR bits, template, detector mask, detectors held)."""
        import torch
        nd = self.n_detectors
        w = np.ascontiguousarray(np.asarray(window, dtype=np.int32).reshape(nd, nd))
        if triggers is None:
            triggers = self.new_peaks()
        if events is None:
            events = torch.empty(self.n_banks * 4, dtype=torch.int32, device="cuda")
        ptr = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None)
        L.check(self.lib.lloid_coincidence(self.handle, ptr(prev), ptr(peaks), int(overlap),
                                           w.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ptr(triggers),
                                           ptr(events), _stream_handle(stream)), "lloid_coincidence")
        return triggers, events

    def events_view(self, events) -> list:
        """Per bank (template, network SNR, detector mask, detectors held);
        template -1 when the bank has no event."""
        raw = events.view(-1, 4).cpu().numpy()
        snr = raw[:, 0].copy().view(np.float32)
        return [(int(r[1]), float(s), int(np.uint32(r[2])), int(r[3])) for r, s in zip(raw, snr)]

    # ------------------------------------------------------------ gradient
    def slice_shapes(self):
        """(2M, L, N) of every slice, banks in order."""
        out = []
        for b, bank in enumerate(self._banks_meta):
            for L_, N_ in bank:
                out.append((2 * self.bank_templates[b], L_, N_))
        return out

    def grad(self, strain, target, stream=None):
        """Loss and gradient of sum (rho - target)^2 over the segment.
        strain: cuda float32 [n_det, T F]; target: cuda float32
        [T, series_floats].  Returns (loss, [dW^s], [dU^s]) with views
        [2M, L] and [L, N] per slice into two packed device tensors."""
        import torch
        T = strain.shape[1] // self.sample_rate
        assert strain.is_cuda and strain.dtype == torch.float32 and strain.is_contiguous()
        assert tuple(target.shape) == (T, self.series_floats) and target.is_contiguous()
        shapes = self.slice_shapes()
        dW = torch.empty(sum(r * l for r, l, _ in shapes), dtype=torch.float32, device="cuda")
        dU = torch.empty(sum(l * n for _, l, n in shapes), dtype=torch.float32, device="cuda")
        loss = ctypes.c_double()
        L.check(self.lib.lloid_grad(self.handle, ctypes.c_void_p(strain.data_ptr()), T,
                                    ctypes.c_void_p(target.data_ptr()), ctypes.byref(loss),
                                    ctypes.c_void_p(dW.data_ptr()), ctypes.c_void_p(dU.data_ptr()),
                                    _stream_handle(stream)), "lloid_grad")
        gw, gu, ow, ou = [], [], 0, 0
        for r, l, n in shapes:
            gw.append(dW[ow:ow + r * l].view(r, l))
            gu.append(dU[ou:ou + l * n].view(l, n))
            ow += r * l
            ou += l * n
        return float(loss.value), gw, gu

    def set_slice(self, index: int, U, W, stream=None) -> None:
        """Replace slice `index` with cuda float64 U [L, N] and W [2M, L]."""
        import torch
        assert U.is_cuda and W.is_cuda and U.dtype == torch.float64 and W.dtype == torch.float64
        L.check(self.lib.lloid_set_slice(self.handle, index, ctypes.c_void_p(U.contiguous().data_ptr()),
                                         ctypes.c_void_p(W.contiguous().data_ptr()), _stream_handle(stream)),
                "lloid_set_slice")

    # ------------------------------------------------------------ timing
    def profile(self, enable: bool = True) -> None:
        """Start (or stop) per-kernel HIP-event timing of push()."""
        L.check(self.lib.lloid_profile_enable(self.handle, 1 if enable else 0), "lloid_profile_enable")

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} since profile(True)."""
        out = {}
        for k, name in enumerate(L.KERNEL_NAMES):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            L.check(self.lib.lloid_profile_read(self.handle, k, ctypes.byref(ms), ctypes.byref(n)),
                    "lloid_profile_read")
            out[name] = (float(ms.value), int(n.value))
        return out

    # ------------------------------------------------------------ state
    def reset(self, stream=None) -> None:
        L.check(self.lib.lloid_reset(self.handle, _stream_handle(stream)), "lloid_reset")

    def state_save(self, stream=None) -> bytes:
        n = ctypes.c_size_t()
        L.check(self.lib.lloid_state_size(self.handle, ctypes.byref(n)), "lloid_state_size")
        buf = ctypes.create_string_buffer(n.value)
        L.check(self.lib.lloid_state_save(self.handle, buf, n.value, _stream_handle(stream)), "lloid_state_save")
        return buf.raw

    def state_load(self, blob: bytes, stream=None) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        L.check(self.lib.lloid_state_load(self.handle, buf, len(blob), _stream_handle(stream)), "lloid_state_load")

    def inspect(self, what: int, index: int, det: int, m_lo: int, m_hi: int, rows: int = 1, stream=None):
        out = np.empty((rows, m_hi - m_lo), dtype=np.float32)
        L.check(self.lib.lloid_inspect(self.handle, what, index, det, m_lo, m_hi,
                                       out.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream)),
                "lloid_inspect")
        return out

    def downsampled(self, D: int, det: int, m_lo: int, m_hi: int) -> np.ndarray:
        return self.inspect(L.INSPECT_DOWNSAMPLED, D, det, m_lo, m_hi)[0]

    def basis_out(self, slice_index: int, n_basis: int, det: int, m_lo: int, m_hi: int) -> np.ndarray:
        return self.inspect(L.INSPECT_BASIS_OUT, slice_index, det, m_lo, m_hi, rows=n_basis)


def svd_basis(H, rank: int, start, iters: int = 200, stream=None):
    """Rank-`rank` truncation of a slice's template matrix H (cuda float64
    [rows, N]) on the GPU (lloid_svd_basis): returns (U [rank, N],
    orthonormal rows spanning the top right singular subspace, and
    W = H U^T [rows, rank]).  start: cuda float64 [rank, N] starting rows
    (seeded Gaussian, say)."""
    import torch
    assert H.is_cuda and H.dtype == torch.float64 and tuple(start.shape) == (rank, H.shape[1])
    H = H.contiguous()
    U = start.detach().clone().contiguous()
    W = torch.empty((H.shape[0], rank), dtype=torch.float64, device="cuda")
    L.check(L.load().lloid_svd_basis(ctypes.c_void_p(H.data_ptr()), H.shape[0], H.shape[1], rank, iters,
                                     ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(W.data_ptr()),
                                     _stream_handle(stream)), "lloid_svd_basis")
    return U, W


def quantize_fp8_rows(U, stream=None):
    """The FP8 form's basis values for U (cuda float64 [L, N]) as a new
    cuda float64 tensor (lloid_quantize_fp8_rows)."""
    import torch
    assert U.is_cuda and U.dtype == torch.float64 and U.dim() == 2
    U = U.contiguous()
    out = torch.empty_like(U)
    L.check(L.load().lloid_quantize_fp8_rows(ctypes.c_void_p(U.data_ptr()), U.shape[0], U.shape[1],
                                             ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
            "lloid_quantize_fp8_rows")
    return out


def orthonormalize(U, W, stream=None) -> None:
    """FP64 CholeskyQR2 on the device, in place: U (cuda float64 [L, N])
    gets orthonormal rows and W (cuda float64 [rows, L]) is updated so that
    W U is unchanged."""
    import torch
    assert U.is_cuda and W.is_cuda and U.dtype == torch.float64 and W.dtype == torch.float64
    assert U.is_contiguous() and W.is_contiguous() and W.shape[1] == U.shape[0]
    lib = L.load()
    L.check(lib.lloid_orthonormalize(ctypes.c_void_p(U.data_ptr()), U.shape[0], U.shape[1],
                                     ctypes.c_void_p(W.data_ptr()), W.shape[0], _stream_handle(stream)),
            "lloid_orthonormalize")


def orthonormalize_noalloc(U, W, info=None, stream=None) -> None:
    """orthonormalize() through lloid_orthonormalize_noalloc: no device
    allocation and no synchronisation (the work is only enqueued; the
    library's static scratch array holds the Gram matrix).  `info`, if
    given, is a cuda int32 tensor of 2 that receives per pass 0 or the
    first failing column + 1."""
    import torch
    assert U.is_cuda and W.is_cuda and U.dtype == torch.float64 and W.dtype == torch.float64
    assert U.is_contiguous() and W.is_contiguous() and W.shape[1] == U.shape[0]
    if info is not None:
        assert info.is_cuda and info.dtype == torch.int32 and info.numel() >= 2
    lib = L.load()
    L.check(lib.lloid_orthonormalize_noalloc(ctypes.c_void_p(U.data_ptr()), U.shape[0], U.shape[1],
                                             ctypes.c_void_p(W.data_ptr()), W.shape[0],
                                             ctypes.c_void_p(info.data_ptr() if info is not None else None),
                                             _stream_handle(stream)),
            "lloid_orthonormalize_noalloc")


class Whitener:
    """PSD estimation and whitening with frequency-domain downsampling for
    n_detectors streams (lloid_whitener_*): push() takes H = block/2 - pad
    new samples per detector and returns H / decimation whitened ones."""

    def __init__(self, n_detectors: int, block: int, pad: int, decimation: int = 1, n_med: int = 7,
                 n_avg: int = 64, stream=None):
        self.lib = L.load()
        self.n_detectors, self.block, self.pad, self.decimation = n_detectors, block, pad, decimation
        self.hop = block // 2 - pad
        self.hop_out = self.hop // decimation
        self.bins = block // decimation // 2 + 1
        cfg = L.WhitenConfig(n_detectors, block, pad, decimation, n_med, n_avg)
        handle = ctypes.c_void_p()
        L.check(self.lib.lloid_whitener_create(ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(handle)),
                "lloid_whitener_create")
        self.handle = handle

    def push(self, x, gap_mask: int = 0, out=None, stream=None):
        """x: cuda float32 [n_det, hop]; returns cuda float32 [n_det, hop_out]."""
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        assert tuple(x.shape) == (self.n_detectors, self.hop)
        if out is None:
            out = torch.empty((self.n_detectors, self.hop_out), dtype=torch.float32, device="cuda")
        L.check(self.lib.lloid_whitener_push(self.handle, ctypes.c_void_p(x.data_ptr()), int(gap_mask),
                                             ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
                "lloid_whitener_push")
        return out

    def psd(self, stream=None):
        import torch
        out = torch.empty((self.n_detectors, self.bins), dtype=torch.float32, device="cuda")
        L.check(self.lib.lloid_whitener_psd(self.handle, ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
                "lloid_whitener_psd")
        return out

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.lloid_whitener_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
