"""The N = 2048 range stage (N' = 4N, N_cp <= N/4, FP32): each length-2048
transform computed as two length-1024 halves (tap parity forward, output
parity inverse), one wave per Doppler row.  Against the FP64 oracle through
the C ABI at the FP32 bound of 1e-5 normwise, with the peak search exact on
the kernel's own P.  Cases cover each window, ragged and extreme N_cp, strided
rows with several frames per call and Doppler padding factors, input scales
far from 1, a noiseless frame, the cells at the transform boundaries, and
batch jobs (P row pointers from the job table) equal to the frames alone."""

import numpy as np
import pytest

from oracle import radar_oracle as O
from synth import frames as S
from tests.gpu_util import check_topk_property, normwise_error, rounded, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
radar = pytest.importorskip("paper_2209_03883_amd.radar")

N = 2048
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    radar.lib()


def _spec(m, ncp, snr=10.0, n_targets=3):
    return S.FrameSpec(n_sub=N, n_sym=m, qam=16, zc_root=7, n_targets=n_targets, snr_db=snr, on_grid=False,
                       rho_min=1.0, rho_max=max(ncp - 1.0, 1.5), nu_abs_max=m / 2 - 1, rayleigh=True, min_sep=2.0)


def _oracle(Y, A, cfg):
    return O.frame_periodogram(rounded(Y), rounded(A), n_pad=cfg.n_pad, m_pad=cfg.m_pad, n_cp=cfg.n_cp,
                               window_kind=cfg.window, zc_root=cfg.zc_root)


def _device(Y, A, cfg, ld):
    F = Y.shape[0]
    if ld is None:
        return torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda()
    Yd = torch.zeros((F, cfg.n_sym, ld), dtype=torch.complex64, device="cuda")
    Ad = torch.zeros_like(Yd)
    Yd[:, :, :N] = torch.from_numpy(Y).cuda()
    Ad[:, :, :N] = torch.from_numpy(A).cuda()
    return Yd[:, :, :N], Ad[:, :, :N]


def _check(Y, A, cfg, label, k=4, ld=None):
    """Y, A: (F, M, N) complex64 host arrays; P against the oracle frame by frame."""
    F = Y.shape[0]
    Yd, Ad = _device(Y, A, cfg, ld)
    P, peaks, n_peaks, status = radar.frame_process(Yd, Ad, cfg, k)
    torch.cuda.synchronize()
    assert int(status.abs().max().cpu()) == 0
    Pn = P.cpu().numpy()
    pk = radar.unpack_peaks(peaks, n_peaks.cpu())
    errs = []
    for f in range(F):
        ref = _oracle(Y[f], A[f], cfg)
        err = normwise_error(Pn[f], ref)
        errs.append(err)
        assert err <= TOL, (label, f, err)
        # the four phases of every range cell, at the transform boundaries:
        # first and last cells of each half of the row, of both parities
        cols = np.array([0, 1, 2, 3, 4, 5, 6, 7, 4 * 1023, 4 * 1023 + 3, 4 * 1024, 4 * 1024 + 1, 4 * 1025 + 2,
                         4 * 2046, 4 * 2047, 4 * 2047 + 3])
        got, want = Pn[f][:, cols], ref[:, cols]
        scale = np.abs(ref).max()
        assert np.max(np.abs(got - want)) <= 2e-5 * scale, (label, f)
        assert check_topk_property(Pn[f], pk[f], k) is None, (label, f)
    say(f"{label}: normwise P error {max(errs):.2e}")


@pytest.mark.parametrize("window", [radar.WIN_RECT, radar.WIN_HANN, radar.WIN_HAMMING])
def test_wide_windows(window):
    cfg = radar.Config(N, 32, 4 * N, 128, 512, zc_root=7, window=window)
    Y, A = S.frames_to_complex64([S.make_frame(_spec(32, 512), 80, window)])
    _check(Y, A, cfg, f"N = 2048, window {window}")


@pytest.mark.parametrize("ncp", [1, 2, 300, 511, 512])
def test_wide_tap_counts(ncp):
    cfg = radar.Config(N, 16, 4 * N, 64, ncp, zc_root=7, window=radar.WIN_HANN)
    Y, A = S.frames_to_complex64([S.make_frame(_spec(16, ncp), 81, ncp)])
    _check(Y, A, cfg, f"N = 2048, n_cp {ncp}")


def test_wide_frames_strided_and_padding():
    # three frames in one call, rows 2100 elements apart, Doppler padded 8x
    cfg = radar.Config(N, 16, 4 * N, 128, 384, zc_root=7, window=radar.WIN_HAMMING)
    Y, A = S.frames_to_complex64([S.make_frame(_spec(16, 384, snr=0.0), 82, i) for i in range(3)])
    _check(Y, A, cfg, "N = 2048, 3 frames, ld 2100, M'/M = 8", ld=2100)


@pytest.mark.parametrize("scale", [1e-18, 1e12])
def test_wide_input_scale(scale):
    cfg = radar.Config(N, 16, 4 * N, 64, 512, zc_root=7, window=radar.WIN_HANN)
    Y, A = S.frames_to_complex64([S.make_frame(_spec(16, 512), 83, 0)])
    _check((Y * np.float32(scale)).astype(np.complex64), A, cfg, f"N = 2048, input scale {scale:g}")


def test_wide_noiseless_single_target():
    spec = _spec(32, 512, n_targets=1)
    spec.noise = False
    cfg = radar.Config(N, 32, 4 * N, 128, 512, zc_root=7, window=radar.WIN_HANN)
    Y, A = S.frames_to_complex64([S.make_frame(spec, 84, 0)])
    _check(Y, A, cfg, "N = 2048, noiseless single target", k=1)


def test_wide_batch_jobs_equal_frames_alone():
    cfg = radar.Config(N, 64, 4 * N, 256, 512, zc_root=7, window=radar.WIN_HANN)
    frames = [S.make_frame(_spec(64, 512, snr=5.0), 85, i) for i in range(3)]
    Y, A = S.frames_to_complex64(frames)
    Yd, Ad = torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda()
    P0, pk0, n0, _ = radar.frame_process(Yd, Ad, cfg, 4)
    b = radar.Batch([(Yd[f], Ad[f], cfg, 4) for f in range(3)], graph=True)
    for _ in range(2):
        b.launch()
        torch.cuda.synchronize()
        for f in range(3):
            assert torch.equal(b.P[f], P0[f]), f
            n = int(n0[f])
            assert int(b.n_peaks[f][0]) == n
            assert torch.equal(b.peaks[f][:n], pk0[f, :n]), f
    say("N = 2048 batch jobs equal the frames alone")
