"""Peaks without a materialised periodogram (radar_frame_process with P =
NULL) against the same call with P written, through the C ABI.

With P NULL the range stage keeps only its row maxima and the peak search
recomputes the listed rows and their neighbours (each row once per run of
listed rows) with the range stage's own row code.  That code is compiled into two kernels, and the compiler may order
a few multiply-adds differently in each, so a recomputed cell can differ from
the written one by a few FP32 ulps.  The rule: the same counts and status, the
same cells rank by rank except at near-ties of the materialised P (the
tolerance the oracle comparisons use), and values within 8 ulps.  At N = 1024
the split matrix-core forms write P with the two-pass 32-point range kernel,
whose row code peaks-only does not use; there the two runs agree to the
forms' error instead.  The small workload is also checked against the FP64
oracle.

The FP16 form (N = 1024) keeps its matrix-core row maxima and rescans the
listed rows in FP32, so its peaks are held to the FP32 run with P written by
the same rule.  The second listing (rows the first one's k-th candidate shows
can still hold a top-k peak) is exercised by cutting the first listing short
with RADAR_PEAKS_ONLY_FIRST_ROWS: the result must not change.
"""

import dataclasses

import numpy as np
import pytest

from oracle import radar_oracle as O
from synth import frames as S
from tests.gpu_util import compare_peak_indices, oracle_ranked, rounded, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
radar = pytest.importorskip("paper_2209_03883_amd.radar")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    radar.lib()


def _both(frames, cfg, k, cfg_peaks_only=None):
    """The frames with P written (cfg) and peaks only (cfg_peaks_only, else cfg)."""
    Y, A = S.frames_to_complex64(frames)
    Yd, Ad = torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda()
    P, pk1, n1, st1 = radar.frame_process(Yd, Ad, cfg, k)
    P0, pk0, n0, st0 = radar.frame_process(Yd, Ad, cfg_peaks_only or cfg, k, materialise=False)
    torch.cuda.synchronize()
    assert P0 is None
    return P.cpu().numpy(), radar.unpack_peaks(pk1, n1.cpu()), st1.cpu().numpy(), \
        radar.unpack_peaks(pk0, n0.cpu()), st0.cpu().numpy()


def _same(res, label, split=False):
    """split: the materialised run took the matrix-core range kernel (N = 1024
    in a split form) while peaks-only recomputes rows with the radix-16 form's
    row code, so the two differ by the forms' error (normwise about 1e-5), not
    by ulps: cells may then swap only at near-ties of 1e-3 relative and values
    agree within 1e-4 of the frame's largest peak."""
    P, with_p, st1, without_p, st0 = res
    np.testing.assert_array_equal(st0, st1, err_msg=label)
    m_pad = P.shape[1]
    exact = 0
    for f in range(P.shape[0]):
        a, b = with_p[f], without_p[f]
        assert len(a) == len(b), (label, f, len(a), len(b))
        ref = [(s, r, float(P[f, s + m_pad // 2, r])) for s, r, *_ in a]
        assert compare_peak_indices([(s, r) for s, r, *_ in b], ref, P[f].astype(np.float64),
                                    near_tie=1e-3 if split else 1e-5) is not None, (label, f, a, b)
        top = max(p for _, _, p, *_ in a) if a else 0.0
        for (s1, r1, p1, *o1), (s0, r0, p0, *o0) in zip(a, b):
            if (s1, r1) == (s0, r0):
                if split:
                    assert abs(p0 - p1) <= 1e-4 * top, (label, f, s1, r1, p1, p0)
                else:
                    assert abs(p0 - p1) <= 8 * np.spacing(np.float32(p1)), (label, f, s1, r1, p1, p0)
                np.testing.assert_allclose(o0, o1, atol=1e-4)
                exact += p0 == p1
    say(f"{label}: {exact} of {sum(len(x) for x in with_p)} peak values bit-identical")


def test_small_workload_peaks_only():
    frames = [S.make_frame(S.spec_small(snr_db=snr), 7, i) for i, snr in enumerate((0.0, -10.0, 10.0, 0.0))]
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1)
    say("peaks only, small workload")
    res = _both(frames, cfg, 3)
    _same(res, "small")
    pk = res[3]
    for f, frame in enumerate(frames):
        P_ref = O.frame_periodogram(rounded(frame.Y), rounded(frame.A), n_pad=1024, m_pad=256, n_cp=32,
                                    window_kind=cfg.window, zc_root=1)
        assert compare_peak_indices([(s, r) for s, r, *_ in pk[f]], oracle_ranked(O, P_ref, 3), P_ref) is not None


# (N, M, N_cp, k, flags): every x4p shape, ragged N_cp, k up to 64, both
# output orders of the range kernel and every precision form
SHAPES = [
    (256, 128, 50, 16, {}),
    (512, 64, 128, 8, {}),
    (512, 256, 97, 64, {}),
    (1024, 256, 256, 8, {}),
    (1024, 128, 200, 8, dict(precision=radar.FLAG_BF16X3)),
    (1024, 128, 256, 8, dict(precision=radar.FLAG_FP16X3)),
    (256, 64, 64, 8, dict(precision=radar.FLAG_BF16X3)),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{s[0]}x{s[1]}-cp{s[2]}-k{s[3]}-{len(s[4])}" for s in SHAPES])
def test_peaks_only_matches_materialised(shape):
    n, m, n_cp, k, extra = shape
    spec = S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=3, n_targets=6, snr_db=-5.0, on_grid=False,
                       rho_min=0.0, rho_max=n_cp - 1.0, nu_abs_max=m / 2 - 1, rayleigh=True, min_sep=1.5)
    frames = [S.make_frame(spec, 81, i) for i in range(3)]
    cfg = radar.Config(n, m, 4 * n, 2 * m, n_cp, zc_root=3, **extra)
    say(f"peaks only {shape}")
    _same(_both(frames, cfg, k), str(shape), split=n == 1024 and bool(extra))


def test_full_frames_peaks_only():
    frames = [S.make_frame(S.spec_full(snr_db=snr), 2, i) for i, snr in enumerate((0.0, -20.0))]
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7)
    say("peaks only, full frames")
    _same(_both(frames, cfg, 8), "full")


def test_every_row_listed():
    # noiseless, one target: fewer than k rows hold a row-profile peak, so the
    # bound is -inf and every row is recomputed and scanned
    spec = dataclasses.replace(S.spec_small(), n_targets=1, noise=False)
    frames = [S.make_frame(spec, 9, i) for i in range(2)]
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1)
    say("peaks only, every row listed")
    _same(_both(frames, cfg, 64), "all rows")


def test_peaks_only_with_threshold_and_refinement():
    frames = [S.make_frame(S.spec_small(snr_db=snr), 8, i) for i, snr in enumerate((-10.0, 5.0))]
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1, threshold=True, pfa=1e-3, noise_power=1.0, refine=True)
    say("peaks only, threshold and refinement")
    _same(_both(frames, cfg, 8), "threshold+refine")


def test_unsupported_shape_is_refused():
    frames = [S.make_frame(S.spec_small(), 7, 0)]
    Y, A = S.frames_to_complex64(frames)
    cfg = radar.Config(256, 64, 2048, 256, 32, zc_root=1)  # N' = 8N
    with pytest.raises(radar.RadarError) as ei:
        radar.frame_process(torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda(), cfg, 3, materialise=False)
    assert ei.value.code == radar.RADAR_E_UNSUPPORTED


@pytest.mark.parametrize("n, m, ncp", [(256, 64, 32), (1024, 128, 256)])
def test_kth_peak_at_the_bound(n, m, ncp):
    # exactly k noiseless targets, each alone in its rows: the k-th largest
    # row-profile peak, the bound tau, is the k-th peak itself.  The recomputed
    # value of that cell may land a few ulps below the range kernel's; the
    # lowered bound must still find it, so every frame reports k peaks
    k = 6
    spec = S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=3, n_targets=k, snr_db=0.0, on_grid=False,
                       rho_min=1.0, rho_max=ncp - 2.0, nu_abs_max=m / 2 - 2, rayleigh=True, min_sep=4.0, noise=False)
    frames = [S.make_frame(spec, 83, i) for i in range(8)]
    cfg = radar.Config(n, m, 4 * n, 4 * m, ncp, zc_root=3)
    say(f"peaks only, k-th peak at the bound, {n}x{m}")
    res = _both(frames, cfg, k)
    for f in range(len(frames)):
        assert len(res[3][f]) == k, (f, res[3][f])
    _same(res, f"k-th at tau {n}x{m}")


# ------------------------------------------------- the FP16 form, peaks only
def _fp16(cfg):
    return dataclasses.replace(cfg, precision=radar.FLAG_FP16)


@pytest.mark.parametrize("m, ncp, k, snr", [(128, 256, 8, -5.0), (64, 100, 16, 0.0), (256, 1, 4, 10.0)])
def test_fp16_peaks_only_matches_fp32(m, ncp, k, snr):
    # the FP16 form's row maxima choose the rows, FP32 rescans them: the
    # peaks are the FP32 periodogram's
    spec = S.FrameSpec(n_sub=1024, n_sym=m, qam=16, zc_root=3, n_targets=6, snr_db=snr, on_grid=False,
                       rho_min=0.0, rho_max=ncp - 1.0, nu_abs_max=m / 2 - 1, rayleigh=True, min_sep=1.5)
    frames = [S.make_frame(spec, 85, i) for i in range(3)]
    cfg = radar.Config(1024, m, 4096, 4 * m, ncp, zc_root=3)
    say(f"FP16 peaks only against FP32 with P, 1024x{m} cp{ncp} k{k}")
    _same(_both(frames, cfg, k, _fp16(cfg)), f"fp16 1024x{m}")


def test_fp16_peaks_only_full_frames():
    frames = [S.make_frame(S.spec_full(snr_db=snr), 2, i) for i, snr in enumerate((0.0, -20.0))]
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7)
    say("FP16 peaks only, full frames")
    _same(_both(frames, cfg, 8, _fp16(cfg)), "fp16 full")


def test_fp16_kth_peak_at_the_bound():
    # as test_kth_peak_at_the_bound, with the FP16 form's maxima choosing the
    # rows: they may miss the FP32 k-th peak by the form's error, which the
    # second listing covers
    k = 6
    spec = S.FrameSpec(n_sub=1024, n_sym=128, qam=16, zc_root=3, n_targets=k, snr_db=0.0, on_grid=False,
                       rho_min=1.0, rho_max=254.0, nu_abs_max=62.0, rayleigh=True, min_sep=4.0, noise=False)
    frames = [S.make_frame(spec, 83, i) for i in range(8)]
    cfg = radar.Config(1024, 128, 4096, 512, 256, zc_root=3)
    say("FP16 peaks only, k-th peak at the bound")
    res = _both(frames, cfg, k, _fp16(cfg))
    for f in range(len(frames)):
        assert len(res[3][f]) == k, (f, res[3][f])
    _same(res, "fp16 k-th at tau")


@pytest.mark.parametrize("first_rows", [2, 8])
@pytest.mark.parametrize("fp16", [False, True])
def test_second_listing_finds_the_rest(monkeypatch, first_rows, fp16):
    # the first listing cut to the rows with the largest maxima (fewer than k
    # of them, or about k): the second one must list every row that can still
    # hold a top-k peak, so the peaks are those of the full listing, bit for bit
    spec = S.FrameSpec(n_sub=1024, n_sym=128, qam=16, zc_root=3, n_targets=6, snr_db=-5.0, on_grid=False,
                       rho_min=0.0, rho_max=255.0, nu_abs_max=63.0, rayleigh=True, min_sep=1.5)
    frames = [S.make_frame(spec, 87, i) for i in range(3)]
    cfg = radar.Config(1024, 128, 4096, 512, 256, zc_root=3)
    cfg0 = _fp16(cfg) if fp16 else cfg
    k = 12
    Y, A = S.frames_to_complex64(frames)
    Yd, Ad = torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda()
    _, pk_full, n_full, _ = radar.frame_process(Yd, Ad, cfg0, k, materialise=False)
    monkeypatch.setenv("RADAR_PEAKS_ONLY_FIRST_ROWS", str(first_rows))
    say(f"second listing after the top {first_rows} rows, fp16={fp16}")
    res = _both(frames, cfg, k, cfg0)
    torch.cuda.synchronize()
    full = radar.unpack_peaks(pk_full, n_full.cpu())
    for f in range(len(frames)):
        assert [p[:2] for p in res[3][f]] == [p[:2] for p in full[f]], (f, res[3][f], full[f])
        assert [p[2] for p in res[3][f]] == [p[2] for p in full[f]], f
    _same(res, f"second listing {first_rows} fp16={fp16}")


def test_fp16_row_maxima_within_the_slack():
    # the listings take the FP16 form's row maxima to be within 1/32 (relative)
    # of the FP32 rows' maxima.  The form's P holds exactly the values whose
    # maxima its store-free kernel keeps (the same products, scaled alike), so
    # the bound is checked here on every row of P, with a wide margin
    specs = [S.spec_full(snr_db=snr) for snr in (-20.0, 0.0, 10.0)]
    specs.append(dataclasses.replace(S.spec_full(), noise=False, n_targets=2))
    frames = [S.make_frame(sp, 89, i) for i, sp in enumerate(specs)]
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7)
    Y, A = S.frames_to_complex64(frames)
    Yd, Ad = torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda()
    worst = 0.0
    for f in range(len(frames)):
        P32, _, _, _ = radar.frame_process(Yd[f:f + 1], Ad[f:f + 1], cfg, 8)
        m32 = P32[0].amax(dim=1).double()
        del P32
        P16, _, _, _ = radar.frame_process(Yd[f:f + 1], Ad[f:f + 1], _fp16(cfg), 8)
        m16 = P16[0].amax(dim=1).double()
        del P16
        big = m32 > m32.max() * 1e-30  # rows that are not numerically zero
        rel = ((m32 - m16).abs() / m32.clamp_min(1e-300))[big]
        worst = max(worst, float(rel.max()))
    say(f"FP16 row maxima: largest relative difference {worst:.2e} (bound 1/32)")
    assert worst <= (1.0 / 32) / 4, worst


def test_fp16_peaks_only_with_threshold_and_refinement():
    # the refinement reads the taps after the peak search, so the recompute
    # rings take their own workspace region here
    spec = S.FrameSpec(n_sub=1024, n_sym=64, qam=16, zc_root=3, n_targets=5, snr_db=0.0, on_grid=False,
                       rho_min=0.0, rho_max=255.0, nu_abs_max=31.0, rayleigh=True, min_sep=1.5)
    frames = [S.make_frame(spec, 91, i) for i in range(3)]
    cfg = radar.Config(1024, 64, 4096, 256, 256, zc_root=3, threshold=True, pfa=1e-4, noise_power=1.0, refine=True)
    say("FP16 peaks only, threshold and refinement")
    _same(_both(frames, cfg, 8, _fp16(cfg)), "fp16 threshold+refine")
