"""GPU parity of threshold detection (Eq. 18, RADAR_FLAG_THRESHOLD) against the
FP64 oracle, through the C ABI.

The GPU forms eta in FP32 from the taps stage's per-symbol sums of 1/|a|^2
and compares it with FP32 periodogram values; the oracle does both in FP64.
A peak may be kept by one side and not the other only when the oracle's value
at that cell lies within the FP32 error band of eta (the periodogram
tolerance of the frame plus 1e-5 of eta); everything else must agree.
"""

import numpy as np
import pytest

from oracle import radar_oracle as O
from synth import frames as S
from tests.gpu_util import P_TOL_FP32, compare_peak_indices, normwise_error, rounded, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
radar = pytest.importorskip("paper_2209_03883_amd.radar")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    radar.lib()


def _run(frames, cfg, k):
    Y, A = S.frames_to_complex64(frames)
    P, peaks, n_peaks, status = radar.frame_process(torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda(), cfg, k)
    torch.cuda.synchronize()
    return P.cpu().numpy(), radar.unpack_peaks(peaks, n_peaks.cpu()), status.cpu().numpy()


def _oracle(frame, cfg, k):
    P_ref = O.frame_periodogram(rounded(frame.Y), rounded(frame.A), n_pad=cfg.n_pad, m_pad=cfg.m_pad,
                                n_cp=cfg.n_cp, window_kind=cfg.window, zc_root=cfg.zc_root, zc_shift=cfg.zc_shift)
    eta = O.cfar_threshold(rounded(frame.A), cfg.noise_power, cfg.pfa, cfg.window)
    half = cfg.m_pad // 2
    det = [(row - half, r, v) for row, r, v in O.detect_threshold(P_ref, eta, k)]
    return P_ref, eta, det


def _compare(gpu, det, P_ref, eta, k, label):
    """gpu: [(s, r, p, ...)] kept by the GPU; det: the oracle's detections."""
    band = P_TOL_FP32 * float(P_ref.max()) + 1e-5 * eta
    half = P_ref.shape[0] // 2
    n = min(len(gpu), len(det))
    assert compare_peak_indices([(s, r) for s, r, *_ in gpu[:n]], det[:n], P_ref) is not None, (label, gpu, det)
    for s, r, *_ in gpu[n:]:  # kept by the GPU only: the oracle's value sits at eta
        assert P_ref[s + half, r] >= eta - band, (label, "extra", s, r, P_ref[s + half, r], eta)
    for s, r, v in det[n:]:   # kept by the oracle only: at eta, and the GPU list was not full
        assert v <= eta + band and len(gpu) < k, (label, "missing", s, r, v, eta)
    for s, r, p, *_ in gpu:   # every kept value at or above eta (to FP32)
        assert p >= eta - band, (label, s, r, p, eta)
    return len(gpu)


@pytest.mark.parametrize("pfa", [1e-2, 1e-3, 1e-6])
@pytest.mark.parametrize("snr_db", [0.0, -20.0])
def test_small_workload_threshold_matches_oracle(pfa, snr_db):
    k = 64
    frames = [S.make_frame(S.spec_small(snr_db=snr_db), 1, i) for i in range(3)]
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1, window=radar.WIN_HANN, threshold=True, pfa=pfa,
                       noise_power=10.0 ** (-snr_db / 10.0))
    say(f"threshold, small workload, snr {snr_db} dB, pfa {pfa:g}")
    P, pk, st = _run(frames, cfg, k)
    counts = []
    for f, frame in enumerate(frames):
        assert st[f] == 0
        P_ref, eta, det = _oracle(frame, cfg, k)
        assert normwise_error(P[f], P_ref) <= P_TOL_FP32
        counts.append(_compare(pk[f], det, P_ref, eta, k, f"frame {f}"))
        # the three targets always pass: a kept peak at each target's cell (at
        # -20 dB per element noise may move the local maximum to a neighbour)
        reach = 0 if snr_db >= 0.0 else 1
        for r0, v0 in zip(frame.rho, frame.nu):
            d = min(max(abs(int(v0 * 4) - s), abs(int(r0 * 4) - r)) for s, r, *_ in pk[f])
            assert d <= reach, (f, r0, v0, d)
    say(f"detections per frame {counts} (oracle {[len(_oracle(fr, cfg, k)[2]) for fr in frames]})")
    # the list is cut by eta, not by k
    assert all(3 <= c < k for c in counts)
    if pfa == 1e-6:
        assert counts == [3, 3, 3]


def test_threshold_cut_is_a_prefix_of_the_topk_list():
    frames = [S.make_frame(S.spec_small(snr_db=0.0), 1, i) for i in range(2)]
    base = radar.Config(256, 64, 1024, 256, 32, zc_root=1, window=radar.WIN_HANN)
    thr = radar.Config(256, 64, 1024, 256, 32, zc_root=1, window=radar.WIN_HANN, threshold=True, pfa=1e-3,
                       noise_power=1.0)
    say("threshold list against the plain top-k list")
    P0, pk0, _ = _run(frames, base, 64)
    P1, pk1, _ = _run(frames, thr, 64)
    np.testing.assert_array_equal(P0, P1)
    for f in range(2):
        assert 0 < len(pk1[f]) < len(pk0[f])
        assert pk1[f] == pk0[f][:len(pk1[f])]


def test_threshold_extremes():
    frames = [S.make_frame(S.spec_small(snr_db=0.0), 1, i) for i in range(2)]
    say("threshold extremes")
    # eta far above every cell: no detections
    hi = radar.Config(256, 64, 1024, 256, 32, zc_root=1, threshold=True, pfa=1e-30, noise_power=1e30)
    _, pk, _ = _run(frames, hi, 8)
    assert [len(p) for p in pk] == [0, 0]
    # eta far below: the full top-k list
    lo = radar.Config(256, 64, 1024, 256, 32, zc_root=1, threshold=True, pfa=0.999, noise_power=1e-30)
    base = radar.Config(256, 64, 1024, 256, 32, zc_root=1)
    _, pk_lo, _ = _run(frames, lo, 8)
    _, pk_base, _ = _run(frames, base, 8)
    assert pk_lo == pk_base and [len(p) for p in pk_lo] == [8, 8]


def test_threshold_with_refinement():
    frames = [S.make_frame(S.spec_full(snr_db=-20.0, n_sub=256, n_sym=64, n_targets=4), 3, i) for i in range(2)]
    ref = radar.Config(256, 64, 1024, 256, 64, zc_root=7, window=radar.WIN_HANN, refine=True)
    both = radar.Config(256, 64, 1024, 256, 64, zc_root=7, window=radar.WIN_HANN, refine=True, threshold=True,
                        pfa=1e-4, noise_power=100.0)
    say("threshold with refinement")
    _, pk_r, _ = _run(frames, ref, 16)
    _, pk_b, _ = _run(frames, both, 16)
    for f in range(2):
        assert 0 < len(pk_b[f]) < 16
        assert pk_b[f] == pk_r[f][:len(pk_b[f])]  # the same peaks with the same sub-cell offsets


def test_full_frame_threshold_matches_oracle():
    frame = S.make_frame(S.spec_full(snr_db=-20.0), 2, 0)
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7, window=radar.WIN_HANN, threshold=True, pfa=1e-5,
                       noise_power=100.0)
    k = 64
    say("threshold, full frame 1024 x 1024 -> 4096 x 4096")
    P, pk, st = _run([frame], cfg, k)
    assert st[0] == 0
    P_ref, eta, det = _oracle(frame, cfg, k)
    assert normwise_error(P[0], P_ref) <= P_TOL_FP32
    n = _compare(pk[0], det, P_ref, eta, k, "full")
    say(f"full frame: {n} detections, oracle {len(det)}")
    assert 0 < n < k


def test_batch_jobs_keep_their_own_thresholds():
    # one shape group, a different noise power per job: each job's eta is its own
    frames = [S.make_frame(S.spec_small(snr_db=0.0), 4, i) for i in range(4)]
    noise = [0.25, 1.0, 4.0, 16.0]
    cfgs = [radar.Config(256, 64, 1024, 256, 32, zc_root=1, threshold=True, pfa=1e-3, noise_power=s2)
            for s2 in noise]
    jobs = []
    for f, c in zip(frames, cfgs):
        Y, A = S.frames_to_complex64([f])
        jobs.append((torch.from_numpy(Y[0]).cuda(), torch.from_numpy(A[0]).cuda(), c, 32))
    say("batch with per-job thresholds")
    b = radar.Batch(jobs, graph=True)
    assert len(b.groups()) == 1
    for rep in range(2):
        b.launch()
        torch.cuda.synchronize()
        lens = []
        for i, (f, c) in enumerate(zip(frames, cfgs)):
            P, pk, st = b.results(i)
            _, pk_alone, _ = _run([f], c, 32)
            assert st == 0 and pk == pk_alone[0], (rep, i)
            lens.append(len(pk))
        say(f"replay {rep}: detections per job {lens}")
        assert lens == sorted(lens, reverse=True) and lens[0] > lens[-1]
    b.close()
