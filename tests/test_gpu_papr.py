"""GPU parity of the PAPR of Eq. 25 (radar_papr) against the FP64 oracle, and
the PAPR of the transmitted symbols under no precoding and the two readings
of the Zadoff-Chu precoding (Sec. III-B).  Tolerance: 1e-5 relative per
symbol (an FP32 FFT; the ratio of a maximum to a mean)."""

import dataclasses

import numpy as np
import pytest

from oracle import radar_oracle as O
from synth import frames as S
from tests.gpu_util import rounded, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
radar = pytest.importorskip("paper_2209_03883_amd.radar")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    radar.lib()


@pytest.mark.parametrize("n,m", [(16, 16), (256, 32), (1024, 16), (4096, 16)])
def test_papr_matches_oracle(n, m):
    rng = np.random.default_rng(n)
    A = (rng.standard_normal((2, m, n)) + 1j * rng.standard_normal((2, m, n))).astype(np.complex64)
    A[1, 3] = 0.0                 # an empty symbol: ratio 0
    A[1, 4] = 0.0
    A[1, 4, 7] = 1.0 + 1.0j       # one subcarrier: ratio 1
    say(f"papr {n}x{m}")
    got = radar.papr(torch.from_numpy(A).cuda()).cpu().numpy()
    for f in range(2):
        np.testing.assert_allclose(got[f], O.papr(rounded(A[f])), rtol=1e-5)
    assert got[1, 3] == 0.0 and got[1, 4] == pytest.approx(1.0, rel=1e-6)


def test_papr_of_the_precoding_readings():
    """PAPR of 16-QAM symbols at N = 1024 without precoding, with the diagonal
    reading and with the dense one (the ZC transform of Eq. 24, whose purpose
    in Sec. III-B is PAPR reduction)."""
    n, m = 1024, 256
    base = S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=None)
    rng = S.rng_for(67, 0)
    A = S.qam_symbols(rng, (m, n), 16)
    stats = {}
    for name, spec in (("none", base), ("diag", dataclasses.replace(base, zc_root=7)),
                       ("dense", dataclasses.replace(base, zc_root=7, zc_dense=True))):
        tx = S.transmit_symbols(A, spec).astype(np.complex64)
        p = radar.papr(torch.from_numpy(tx)[None].cuda()).cpu().numpy()[0]
        np.testing.assert_allclose(p, O.papr(rounded(tx)), rtol=1e-5)
        db = 10 * np.log10(p)
        stats[name] = (float(db.mean()), float(np.percentile(db, 99)))
    say("PAPR (dB) mean / 99th percentile: " + ", ".join(f"{k} {v[0]:.2f} / {v[1]:.2f}" for k, v in stats.items()))
    # the dense transform lowers the PAPR well below plain OFDM
    assert stats["dense"][0] < stats["none"][0] - 3.0


@pytest.mark.parametrize("n", [16, 256, 1024, 4096])
def test_hpa_matches_oracle(n):
    m = 16
    rng = np.random.default_rng(n + 1)
    A = (rng.standard_normal((2, m, n)) + 1j * rng.standard_normal((2, m, n))).astype(np.complex64)
    A[1, 2] = 0.0                 # an empty symbol stays empty
    A[1, 3] = 0.0
    A[1, 3, 5] = 2.0 - 1.0j       # a constant envelope: a plain gain
    for q in (0.0, 2.0, 6.0):
        got = radar.hpa(torch.from_numpy(A).cuda(), q).cpu().numpy()
        for f in range(2):
            ref = O.hpa(rounded(A[f]), q)
            err = float(np.max(np.abs(got[f] - ref)) / np.max(np.abs(ref)))
            assert err <= 1e-5, (n, q, f, err)
    say(f"hpa {n}: within 1e-5")


def test_hpa_distortion_under_the_precoding_readings():
    """Eq. 26 at q = 2 dB on 16-QAM at N = 1024: the distortion the radar's LS
    estimate sees (the amplified symbols minus their best scalar fit, divided by
    the known symbols) without precoding and with the two ZC readings."""
    n, m = 1024, 256
    base = S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=None)
    A = S.qam_symbols(S.rng_for(68, 0), (m, n), 16)
    res = {}
    for name, spec in (("none", base), ("diag", dataclasses.replace(base, zc_root=7)),
                       ("dense", dataclasses.replace(base, zc_root=7, zc_dense=True))):
        tx = torch.from_numpy(S.transmit_symbols(A, spec).astype(np.complex64)).cuda()
        out = radar.hpa(tx[None], 2.0)[0].to(torch.complex128)
        t64 = tx.to(torch.complex128)
        alpha = (out * t64.conj()).sum() / (t64.abs() ** 2).sum()
        d = out - alpha * t64
        sdr = float((d.abs() ** 2).sum() / ((alpha * t64).abs() ** 2).sum())
        ls = float(((d / t64).abs() ** 2).mean() / alpha.abs() ** 2)
        res[name] = (10 * np.log10(sdr), 10 * np.log10(ls))
    say("HPA q = 2 dB, distortion (dB) in the symbols / in the LS estimate: "
        + ", ".join(f"{k} {v[0]:.1f} / {v[1]:.1f}" for k, v in res.items()))
    # the low-PAPR waveform leaves the amplifier less distorted (measured 7 dB);
    # what the radar's LS estimate sees is not better for it (division by the
    # near-Gaussian precoded symbols)
    assert res["dense"][0] < res["none"][0] - 5.0
    assert res["dense"][1] > res["none"][1] - 3.0
