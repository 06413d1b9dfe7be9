"""GPU parity of PSD estimation and whitening with frequency-domain
downsampling (Sec. II.B.2) through the C ABI against the FP64 oracle.

Both sides get the same seeded float32 input: white noise on one detector,
red AR(1) noise on the other, gap pushes on one detector, D = 1 and 4, and
the paper's low-latency block (4 s at 16384 Hz, 1 s of padding, D = 4).
Every output sample and the PSD are compared.

Tolerance: the FP32 transforms err by about log2(N) unit roundoffs of the
block's RMS; whitening divides each bin by sqrt(PSD), which scales a bin's
absolute error by sqrt(max PSD / PSD) (10 for the red detector), and the
log-domain running average and the inverse transform add a few roundoffs:
about 1e-5 of the unit output.  The test allows 2e-4 absolute on outputs of
unit variance and 1e-4 relative on the PSD.
"""
import numpy as np
import pytest

import synth
from oracle import lloid as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def whitener_cls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_04730_amd import Whitener
    return Whitener


def _inputs(n_det, n, seed):
    g = synth.rng_for(91, synth.PURPOSE_NOISE, seed)
    x = g.standard_normal((n_det, n))
    for d in range(1, n_det, 2):                    # red noise on odd detectors
        e = x[d].copy()
        for i in range(1, n):
            e[i] = 0.95 * e[i - 1] + x[d, i]
        x[d] = e
    return (3.0 * x).astype(np.float32)


def _compare(whitener_cls, N, Z, D, pushes, gaps=()):
    nd = 2
    w = whitener_cls(nd, N, Z, D)
    H = w.hop
    x = _inputs(nd, pushes * H, N + D)
    refs = [O.Whitener(N, Z, d=D) for _ in range(nd)]
    xs = torch.from_numpy(x).cuda()
    worst = 0.0
    for i in range(pushes):
        mask = 1 if i in gaps else 0
        got = w.push(xs[:, i * H:(i + 1) * H].contiguous(), gap_mask=mask).cpu().numpy()
        for d in range(nd):
            ref = refs[d].push(x[d, i * H:(i + 1) * H].astype(np.float64), gap=(d == 0 and i in gaps))
            err = float(np.abs(got[d] - ref).max())
            worst = max(worst, err)
            assert err <= 2e-4, (i, d, err)
    psd = w.psd().cpu().numpy()
    for d in range(nd):
        rel = np.abs(psd[d] - refs[d].psd) / refs[d].psd
        assert rel.max() <= 1e-4, (d, rel.max())
    print(f"N={N} Z={Z} D={D}: worst output error {worst:.2e}")
    return worst


@pytest.mark.parametrize("D", [1, 4])
def test_whitening_matches_oracle(whitener_cls, D):
    _compare(whitener_cls, 4096, 512, D, 30, gaps=(10, 11))


def test_paper_block_matches_oracle(whitener_cls):
    """4 s blocks at 16384 Hz with 1 s of padding, output at 4096 Hz."""
    _compare(whitener_cls, 65536, 16384, 4, 10)


def test_errors(whitener_cls):
    from paper_2511_04730_amd._lib import LloidError
    for args, status in (((2, 4096, 1025, 1), -2), ((2, 4000, 512, 1), -2), ((2, 4096, 512, 3), -2),
                         ((33, 4096, 512, 1), -1), ((2, 4096, 512, 1, 4), -1)):
        with pytest.raises(LloidError) as e:
            whitener_cls(*args)
        assert e.value.status == status
