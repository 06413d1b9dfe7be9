"""The stored oracle triggers of the batched workload (written by
tests/golden/make_batched_triggers.py) are the oracle's: the file matches
the workload and strain it was made from, and two banks recomputed here give
the same triggers and near-maximum sets."""
import importlib.util
import os

import numpy as np

import synth
from oracle import lloid as O

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _maker():
    spec = importlib.util.spec_from_file_location("mk", os.path.join(HERE, "make_batched_triggers.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    return mk


def test_stored_triggers_are_the_oracles():
    mk = _maker()
    g = np.load(os.path.join(HERE, "batched_triggers_stride64.npz"), allow_pickle=False)
    w = synth.cached_workload("c3", synth.config3)
    x = synth.workload_strain(w, mk.STRIDE + 1)
    np.testing.assert_allclose(g["fingerprint"], mk.fingerprint(w, x), rtol=1e-12)
    count = g["count"]
    assert len(count) == w.n_detectors * w.n_templates
    off = np.concatenate([[0], np.cumsum(count)])
    F = w.sample_rate
    cfg = O.OracleConfig(F)
    # the two smallest banks, both detectors
    sizes = [b.n_templates * sum(s.n_taps for s in b.slices) for b in w.banks]
    start = np.concatenate([[0], np.cumsum([w.n_detectors * b.n_templates for b in w.banks])])
    for b in np.argsort(sizes)[:2]:
        bank = w.banks[b]
        for d in range(w.n_detectors):
            z, _ = O.lloid_filter(x[d, :(mk.STRIDE + 1) * F], bank, cfg, n_strides=1, first_stride=mk.STRIDE)
            mag = np.abs(z)
            for i in range(bank.n_templates):
                t = start[b] + d * bank.n_templates + i
                idx = g["index"][off[t]:off[t + 1]]
                zs = g["re"][off[t]:off[t + 1]] + 1j * g["im"][off[t]:off[t + 1]]
                assert idx[0] == np.argmax(mag[i])
                near = np.nonzero(mag[i] >= mag[i].max() - mk.TAU * max(mag[i].max(), 4.0))[0]
                assert sorted(idx.tolist()) == sorted(near.tolist())
                np.testing.assert_allclose(zs, z[i, idx], rtol=1e-6, atol=1e-6)
