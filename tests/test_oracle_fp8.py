"""Pins of the oracle's e4m3 rounding and FP8 basis values (reading 19),
CPU only: the rounding equals torch's float8_e4m3fn conversion (the OCP
format) on values spanning every binade and the subnormals, fixes every
representable value and takes ties to the even mantissa; each row's scaled
maximum lands in (224, 448]; the row values differ from the basis by at
most half a spacing of the row's binade."""
import numpy as np
import torch

import synth
from oracle import lloid as O


def test_e4m3_rounding_matches_torch():
    g = synth.rng_for(90, synth.PURPOSE_NOISE, 0)
    x = g.uniform(-1, 1, 200000) * 2.0 ** g.uniform(-12, np.log2(448.0), 200000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(O.e4m3_round(x.astype(np.float32)), ref)


def test_representable_values_are_fixed_and_ties_go_to_even():
    vals = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    fin = vals[np.isfinite(vals)]
    assert np.array_equal(O.e4m3_round(fin), fin) and fin.max() == 448.0
    assert O.e4m3_round(np.array([1.0625, 1.1875, 3 * 2.0 ** -10, 2.0 ** -10])).tolist() == [1.0, 1.25, 2.0 ** -8, 0.0]


def test_row_scale_and_error():
    g = synth.rng_for(90, synth.PURPOSE_NOISE, 1)
    U = np.linalg.qr(g.standard_normal((700, 40)))[0].T * g.uniform(0.01, 5.0, (40, 1))
    Q = O.quantize_fp8_rows(U)
    mx = np.abs(U).max(axis=1)
    e = np.floor(np.log2(448.0 / mx))
    assert np.all((mx * 2 ** e > 224) & (mx * 2 ** e <= 448))
    spacing = 2.0 ** (np.clip(np.floor(np.log2(np.abs(U) * 2 ** e[:, None])), -6, 8) - 3) / 2 ** e[:, None]
    assert np.all(np.abs(Q - U) <= 0.5 * spacing * (1 + 1e-6))
    assert np.array_equal(O.quantize_fp8_rows(Q), Q)          # idempotent
