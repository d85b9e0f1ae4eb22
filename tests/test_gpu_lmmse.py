"""GPU parity of the LMMSE-based DFT-CE (per-tap Wiener weights on the kept
taps, Sec. III-A / Fig. 5) against the FP64 oracle, through the C ABI.

The weights are an input to both sides: the library's own host helper
(radar_tap_wiener_weights) computes them from the generator's tap power
profile and the noise per tap, and the oracle is handed the same FP32 values.
"""

import numpy as np
import pytest

from oracle import radar_oracle as O
from synth import frames as S
from tests.gpu_util import P_TOL_FP32, check_topk_property, compare_peak_indices, normwise_error, oracle_ranked, \
    rounded, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
radar = pytest.importorskip("paper_2209_03883_amd.radar")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    radar.lib()


def _weights(spec, n_cp, qam_inv_power):
    """Wiener weights of the kept taps: the generator's prior against
    sigma^2 mean(1/|a|^2) / N of noise per tap."""
    sigma2 = 10.0 ** (-spec.snr_db / 10.0)
    prior = S.tap_power_profile(spec)[:n_cp]
    g = np.asarray(radar.tap_wiener_weights(prior, sigma2 * qam_inv_power / spec.n_sub), dtype=np.float32)
    return g, torch.from_numpy(g).cuda()


def _run(frames, cfg, k):
    Y, A = S.frames_to_complex64(frames)
    P, peaks, n_peaks, status = radar.frame_process(torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda(), cfg, k)
    torch.cuda.synchronize()
    return P.cpu().numpy(), radar.unpack_peaks(peaks, n_peaks.cpu()), status.cpu().numpy()


def _check(P_gpu, pk_gpu, frame, cfg, g, k, label):
    P_ref = O.frame_periodogram(rounded(frame.Y), rounded(frame.A), n_pad=cfg.n_pad, m_pad=cfg.m_pad, n_cp=cfg.n_cp,
                                window_kind=cfg.window, zc_root=cfg.zc_root, tap_weights=g.astype(np.float64))
    err = normwise_error(P_gpu, P_ref)
    say(f"{label}: normwise P error {err:.3e}")
    assert err <= P_TOL_FP32
    assert check_topk_property(P_gpu, pk_gpu, k) is None
    assert compare_peak_indices([(s, r) for s, r, *_ in pk_gpu], oracle_ranked(O, P_ref, k), P_ref) is not None


@pytest.mark.parametrize("snr_db", [-5.0, 10.0])
def test_small_workload_lmmse(snr_db):
    spec = S.spec_small(snr_db=snr_db)
    g, gd = _weights(spec, 32, 1.0)  # QPSK: |a| = 1
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1, tap_weights=gd)
    frames = [S.make_frame(spec, 7, i) for i in range(3)]
    say(f"LMMSE-based DFT-CE, small workload, {snr_db} dB, weights {g.min():.3f}..{g.max():.3f}")
    P, pk, st = _run(frames, cfg, 3)
    for f, frame in enumerate(frames):
        assert st[f] == 0
        _check(P[f], pk[f], frame, cfg, g, 3, f"frame {f}")


# (N, M, N', M', N_cp): both taps kernels, a ragged N_cp, and N_cp = N (LMMSE-based LS-CE)
LMMSE_SHAPES = [
    (64, 32, 256, 64, 16),
    (256, 64, 1024, 256, 256),
    (1024, 16, 4096, 32, 256),
    (2048, 16, 8192, 32, 300),
]


@pytest.mark.parametrize("shape", LMMSE_SHAPES, ids=[f"{s[0]}x{s[1]}-cp{s[4]}" for s in LMMSE_SHAPES])
def test_lmmse_shapes(shape):
    n, m, n_pad, m_pad, n_cp = shape
    spec = S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=3, n_targets=3, snr_db=0.0, on_grid=False, rho_min=0.0,
                       rho_max=min(n_cp, n) - 1.0, nu_abs_max=m / 2 - 1, rayleigh=True, min_sep=1.5)
    frame = S.make_frame(spec, 70, n)
    g, gd = _weights(spec, n_cp, float(np.mean(1.0 / np.abs(rounded(frame.A)) ** 2)))
    cfg = radar.Config(n, m, n_pad, m_pad, n_cp, zc_root=3, tap_weights=gd)
    say(f"LMMSE shape {shape}")
    P, pk, st = _run([frame], cfg, 3)
    assert st[0] == 0
    _check(P[0], pk[0], frame, cfg, g, 3, f"shape {shape}")


def test_unit_weights_equal_plain_dft_ce():
    frames = [S.make_frame(S.spec_small(snr_db=0.0), 7, i) for i in range(2)]
    ones = torch.ones(32, dtype=torch.float32, device="cuda")
    say("unit weights")
    P0, pk0, _ = _run(frames, radar.Config(256, 64, 1024, 256, 32, zc_root=1), 3)
    P1, pk1, _ = _run(frames, radar.Config(256, 64, 1024, 256, 32, zc_root=1, tap_weights=ones), 3)
    np.testing.assert_array_equal(P0, P1)
    assert pk0 == pk1


def test_periodogram_entry_with_weights():
    n, m, n_cp = 256, 64, 48
    rng = np.random.default_rng(12)
    H = (rng.standard_normal((2, m, n)) + 1j * rng.standard_normal((2, m, n))).astype(np.complex64)
    g = rng.uniform(0.0, 1.0, n_cp).astype(np.float32)
    cfg = radar.Config(n, m, 1024, 256, n_cp, zc_root=None, window=radar.WIN_HAMMING,
                       tap_weights=torch.from_numpy(g).cuda())
    say("radar_periodogram with tap weights")
    P = radar.periodogram(torch.from_numpy(H).cuda(), cfg)
    torch.cuda.synchronize()
    P = P.cpu().numpy()
    for i in range(2):
        ref = O.periodogram(O.lmmse_dft_ce(H[i].astype(np.complex128), n_cp, g.astype(np.float64)), 1024, 256,
                            radar.WIN_HAMMING)
        assert normwise_error(P[i], ref) <= P_TOL_FP32


def test_lmmse_batch_matches_frames_alone():
    # one shape, two weight vectors: two groups, each job equal to its frame alone
    spec = S.spec_small(snr_db=-5.0)
    g1, gd1 = _weights(spec, 32, 1.0)
    gd2 = torch.from_numpy(np.sqrt(g1)).cuda()
    jobs, alone = [], []
    for i, gd in enumerate((gd1, gd2, gd1)):
        cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1, tap_weights=gd)
        f = S.make_frame(spec, 71, i)
        Y, A = S.frames_to_complex64([f])
        jobs.append((torch.from_numpy(Y[0]).cuda(), torch.from_numpy(A[0]).cuda(), cfg, 3))
        alone.append(_run([f], cfg, 3))
    say("LMMSE weights in a batch")
    b = radar.Batch(jobs, graph=True)
    assert len(b.groups()) == 2
    b.launch()
    torch.cuda.synchronize()
    for i in range(3):
        P, pk, st = b.results(i)
        assert st == 0
        np.testing.assert_array_equal(P, alone[i][0][0])
        assert pk == alone[i][1][0]
    b.close()
