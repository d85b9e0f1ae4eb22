"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, sizes workspaces, and rejects bad arguments before touching the GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "radar.h")

radar = pytest.importorskip("paper_2209_03883_amd.radar")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(radar_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ("radar_frame_process", "radar_periodogram", "radar_detect_topk"):
        assert want in names


def test_library_exports_every_declared_symbol():
    L = radar.lib()
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert radar.EXPORTED and set(radar.EXPORTED) <= set(_declared_functions())


def test_status_strings():
    assert radar.status_string(0) == "ok"
    assert "coprime" in radar.status_string(radar.RADAR_E_NOT_COPRIME) or \
        "prime" in radar.status_string(radar.RADAR_E_NOT_COPRIME)
    assert radar.status_string(-99) == "unknown status code"


def _ws(cfg, F=1, k=8):
    return radar.lib().radar_frame_workspace_size(ctypes.byref(cfg.desc()), F, k)


def _al(x):
    return (x + 255) // 256 * 256


def _peak_ws(F, m_pad, k):
    # row maxima, tau, row count, second-listing start, row list, per-row candidates
    return (_al(F * m_pad * 4) + _al(F * 4) + _al(F * 4) + _al(F * 4) + _al(F * m_pad * 4)
            + _al(F * m_pad * k * 8))


def test_workspace_size_arithmetic():
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7)
    for F in (1, 3):
        taps = F * 1024 * 256 * 8
        U = F * 4096 * 256 * 8
        assert _ws(cfg, F, 8) == _al(taps) + _al(U) + _peak_ws(F, 4096, 8)
    assert radar.lib().radar_detect_workspace_size(4096, 4096, 2, 8) == _peak_ws(2, 4096, 8)
    # threshold detection adds the per-symbol sums of 1/|a|^2, [F][M] floats
    thr = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7, threshold=True, noise_power=1.0)
    for F in (1, 3):
        assert _ws(thr, F, 8) == _ws(cfg, F, 8) + _al(F * 1024 * 4)


@pytest.mark.parametrize("bad,code", [
    (dict(n_sub=1000), radar.RADAR_E_UNSUPPORTED),     # not a power of two
    (dict(n_sub=8, n_cp=8, n_pad=64), radar.RADAR_E_UNSUPPORTED),  # below the smallest FFT
    (dict(n_sym=8192, m_pad=8192), radar.RADAR_E_UNSUPPORTED),
    (dict(n_pad=512), radar.RADAR_E_ARG),              # N' < N
    (dict(n_pad=16384), radar.RADAR_E_UNSUPPORTED),    # N'/N = 16
    (dict(n_cp=0), radar.RADAR_E_ARG),
    (dict(n_cp=1025), radar.RADAR_E_ARG),
    (dict(window=7), radar.RADAR_E_ARG),
    (dict(zc_root=8), radar.RADAR_E_NOT_COPRIME),      # gcd(8, 1024) != 1
    (dict(n_sym=2048, m_pad=4096, refine=True), radar.RADAR_E_UNSUPPORTED),  # refinement needs M <= 1024
    (dict(n_sym=16, m_pad=512, refine=True), radar.RADAR_E_UNSUPPORTED),     # and M'/M <= 16
])
def test_validation_rejects(bad, code):
    base = dict(n_sub=1024, n_sym=1024, n_pad=4096, m_pad=4096, n_cp=256, zc_root=7)
    base.update(bad)
    cfg = radar.Config(**base)
    L = radar.lib()
    assert L.radar_frame_workspace_size(ctypes.byref(cfg.desc()), 1, 8) == 0
    # radar_frame_process validates before any HIP call: dummy non-null pointers are never touched
    dummy = 256
    rc = L.radar_frame_process(ctypes.byref(cfg.desc()), 1, dummy, dummy, 0, dummy, 0, 8, dummy, dummy,
                               dummy, dummy, 1 << 40, None)
    assert rc == code


def test_process_rejects_bad_pointers_and_workspace():
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1)
    L = radar.lib()
    d = ctypes.byref(cfg.desc())
    need = L.radar_frame_workspace_size(d, 1, 3)
    p = 256
    assert L.radar_frame_process(d, 1, None, p, 0, p, 0, 3, p, p, p, p, need, None) == radar.RADAR_E_ARG
    assert L.radar_frame_process(d, 1, p, p, 0, p + 4, 0, 3, p, p, p, p, need, None) == radar.RADAR_E_ARG  # P misaligned
    assert L.radar_frame_process(d, 1, p, p, 0, p, 0, 0, p, p, p, p, need, None) == radar.RADAR_E_ARG     # k = 0
    assert L.radar_frame_process(d, 1, p, p, 0, p, 0, 65, p, p, p, p, need, None) == radar.RADAR_E_ARG    # k > 64
    assert L.radar_frame_process(d, 1, p, p, 0, p, 0, 3, p, p, p, p, need - 1, None) == radar.RADAR_E_WORKSPACE
    assert L.radar_frame_process(d, 0, p, p, 0, p, 0, 3, p, p, p, p, need, None) == radar.RADAR_E_ARG     # no frames
    # overlapping frames
    assert L.radar_frame_process(d, 2, p, p, 100, p, 1024 * 256, 3, p, p, p, p, 10 * need, None) == radar.RADAR_E_ARG
    # periodogram refuses ZC mode
    assert L.radar_periodogram(d, 1, p, 0, p, 0, p, need, None) == radar.RADAR_E_ARG


def test_noalloc_rejects_before_any_hip_call():
    L = radar.lib()
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7)
    d = ctypes.byref(cfg.desc())
    p = 256
    fs, ps = 1024 * 1024, 4096 * 4096
    # four full frames need more than the library's own workspace
    assert L.radar_frame_workspace_size(d, 4, 8) > (32 << 20) >= L.radar_frame_workspace_size(d, 3, 8)
    assert L.radar_frame_process_noalloc(d, 4, p, p, fs, p, ps, 8, p, p, p, None) == radar.RADAR_E_WORKSPACE
    assert L.radar_frame_process_noalloc(d, 1, p, p, 0, p, 0, 0, p, p, p, None) == radar.RADAR_E_ARG   # k = 0
    assert L.radar_frame_process_noalloc(d, 1, p, p, 0, p + 4, 0, 8, p, p, p, None) == radar.RADAR_E_ARG  # P misaligned
    assert L.radar_frame_process_noalloc(d, 0, p, p, 0, p, 0, 8, p, p, p, None) == radar.RADAR_E_ARG   # no frames


@pytest.mark.parametrize("change, code", [
    (dict(), radar.RADAR_E_WORKSPACE),                                   # supported: reaches the workspace check
    (dict(n_sub=2048, n_cp=256, n_pad=8192), radar.RADAR_E_UNSUPPORTED),  # N > 1024
    (dict(n_pad=2048), radar.RADAR_E_UNSUPPORTED),                       # N' = 8N
    (dict(n_cp=100), radar.RADAR_E_UNSUPPORTED),                         # 4 N_cp > N
    (dict(n_sub=128, n_cp=16, n_pad=512), radar.RADAR_E_UNSUPPORTED),    # N < 256
])
def test_peaks_only_shapes(change, code):
    # P = NULL (peaks only) is validated before any HIP call; a 1-byte
    # workspace stops the supported shape right after the pointer checks
    base = dict(n_sub=256, n_sym=64, n_pad=1024, m_pad=256, n_cp=32, zc_root=1)
    base.update(change)
    cfg = radar.Config(**base)
    L = radar.lib()
    p = 256
    rc = L.radar_frame_process(ctypes.byref(cfg.desc()), 1, p, p, 0, None, 0, 3, p, p, p, p, 1, None)
    assert rc == code
    # the other entry points still need P
    assert L.radar_periodogram(ctypes.byref(radar.Config(**{**base, "zc_root": None}).desc()), 1, p, 0, None, 0, p,
                               1 << 40, None) == radar.RADAR_E_ARG


def test_detect_rejects():
    L = radar.lib()
    p = 256
    assert L.radar_detect_topk(p, 100, 64, 1, 0, 3, p, p, p, 1 << 20, None) == radar.RADAR_E_UNSUPPORTED
    assert L.radar_detect_topk(p, 64, 64, 1, 0, 0, p, p, p, 1 << 20, None) == radar.RADAR_E_ARG
    assert L.radar_detect_topk(p, 64, 64, 1, 0, 3, p, p, p, 10, None) == radar.RADAR_E_WORKSPACE
    assert L.radar_detect_topk(None, 64, 64, 1, 0, 3, p, p, p, 1 << 20, None) == radar.RADAR_E_ARG


def test_flags_validation():
    L = radar.lib()
    d = radar.Config(256, 64, 1024, 256, 32, zc_root=1).desc()
    d.flags = 16  # unknown bit
    assert L.radar_frame_workspace_size(ctypes.byref(d), 1, 3) == 0
    ok = radar.Config(256, 64, 1024, 256, 32, refine=True)
    need = L.radar_frame_workspace_size(ctypes.byref(ok.desc()), 1, 3)
    assert need > 0
    # the periodogram entry finds no peaks: the refine flag is an argument error
    assert L.radar_periodogram(ctypes.byref(ok.desc()), 1, 256, 0, 256, 0, 256, need, None) == radar.RADAR_E_ARG


@pytest.mark.parametrize("pfa,noise,ok", [
    (1e-2, 1.0, True), (1e-6, 1e-9, True), (0.0, 1.0, False), (1.0, 1.0, False), (-0.1, 1.0, False),
    (float("nan"), 1.0, False), (1e-2, 0.0, False), (1e-2, -1.0, False), (1e-2, float("inf"), False),
    (1e-2, float("nan"), False),
])
def test_threshold_validation(pfa, noise, ok):
    L = radar.lib()
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1, threshold=True, pfa=pfa, noise_power=noise)
    assert (L.radar_frame_workspace_size(ctypes.byref(cfg.desc()), 1, 3) > 0) == ok
    # without the flag the two fields are ignored
    cfg.threshold = False
    assert L.radar_frame_workspace_size(ctypes.byref(cfg.desc()), 1, 3) > 0


def test_threshold_rejected_by_periodogram_and_sft():
    L = radar.lib()
    cfg = radar.Config(256, 64, 1024, 256, 32, threshold=True, noise_power=1.0)
    need = L.radar_frame_workspace_size(ctypes.byref(cfg.desc()), 1, 3)
    assert need > 0
    assert L.radar_periodogram(ctypes.byref(cfg.desc()), 1, 256, 0, 256, 0, 256, need, None) == radar.RADAR_E_ARG
    s = radar.sft_desc(8)
    assert L.radar_fps_sft_workspace_size(ctypes.byref(cfg.desc()), ctypes.byref(s), 1) == 0


def test_dense_precoding_validation():
    L = radar.lib()
    ok = radar.Config(256, 64, 1024, 256, 32, zc_root=7, zc_shift=-3, zc_dense=True)
    assert ok.desc().zc_mode == radar.ZC_DENSE
    # 256 <= N <= 1024: the taps kernel folds the precoding in, no extra region
    assert L.radar_frame_workspace_size(ctypes.byref(ok.desc()), 2, 3) == _ws(
        radar.Config(256, 64, 1024, 256, 32), 2, 3)
    # other N: plus the FP64 stage's LS estimate, [F][M][N] complex64
    small = radar.Config(128, 64, 512, 256, 32, zc_root=7, zc_shift=-3, zc_dense=True)
    assert L.radar_frame_workspace_size(ctypes.byref(small.desc()), 2, 3) == (
        _ws(radar.Config(128, 64, 512, 256, 32), 2, 3) + _al(2 * 64 * 128 * 8))
    even = radar.Config(256, 64, 1024, 256, 32, zc_root=4, zc_dense=True)
    d = even.desc()
    assert L.radar_frame_workspace_size(ctypes.byref(d), 1, 3) == 0
    # FPS-SFT gathers single elements: the dense transform is not offered there
    s = radar.sft_desc(8)
    assert L.radar_fps_sft_workspace_size(ctypes.byref(ok.desc()), ctypes.byref(s), 1) == 0
    bad = ok.desc()
    bad.zc_mode = 3
    assert L.radar_frame_workspace_size(ctypes.byref(bad), 1, 3) == 0


def test_tap_wiener_weights_host():
    from oracle import radar_oracle as O

    p = [0.0, 1e-3, 0.5, 2.0, 1e6]
    g = radar.tap_wiener_weights(p, 0.25)
    np.testing.assert_allclose(g, O.wiener_tap_weights(p, 0.25).astype(np.float32), rtol=1e-7)
    assert radar.tap_wiener_weights([0.0, 3.0], 0.0) == [0.0, 1.0]
    L = radar.lib()
    src = (ctypes.c_double * 2)(1.0, -1.0)
    dst = (ctypes.c_float * 2)()
    assert L.radar_tap_wiener_weights(src, 2, 1.0, dst) == radar.RADAR_E_ARG      # negative power
    src = (ctypes.c_double * 2)(1.0, 1.0)
    assert L.radar_tap_wiener_weights(src, 2, -1.0, dst) == radar.RADAR_E_ARG     # negative noise
    assert L.radar_tap_wiener_weights(src, 2, float("nan"), dst) == radar.RADAR_E_ARG
    assert L.radar_tap_wiener_weights(src, 0, 1.0, dst) == radar.RADAR_E_ARG


def test_tap_weights_validation():
    L = radar.lib()
    d = radar.Config(256, 64, 1024, 256, 32, zc_root=1).desc()
    d.tap_weights = 4096 + 2  # misaligned device address (never dereferenced here)
    assert L.radar_frame_workspace_size(ctypes.byref(d), 1, 3) == 0
    d.tap_weights = 4096
    assert L.radar_frame_workspace_size(ctypes.byref(d), 1, 3) > 0
    s = radar.sft_desc(8)
    assert L.radar_fps_sft_workspace_size(ctypes.byref(d), ctypes.byref(s), 1) == 0


@pytest.mark.parametrize("change", [dict(n_sub=100), dict(n_guard=-1), dict(n_guard=65), dict(max_targets=0),
                                    dict(fc_over_df=0.0), dict(fc_over_df=float("inf")), dict(ld=32)])
def test_simulate_validation(change):
    L = radar.lib()
    base = dict(n_sub=64, n_sym=16, n_guard=16, max_targets=4, ld=64, fc_over_df=320833.0)
    d = radar.SimDesc(**{**base, **change})
    rc = L.radar_simulate_frames(ctypes.byref(d), 1, 4096, 0, 4096, 4096, None, 4096, None, None)
    assert rc in (radar.RADAR_E_ARG, radar.RADAR_E_UNSUPPORTED)


def test_sft_default_settings():
    d = radar.sft_desc(8)
    assert (d.n_dirs, d.k, d.flags) == (8, 8, 0)
    assert [tuple(d.dirs[i]) for i in range(8)] == [(1, 1), (1, -1), (1, 2), (2, 1), (1, -2), (2, -1), (1, 0), (0, 1)]
    assert d.pfa == pytest.approx(1e-2) and d.tol == pytest.approx(0.25)


def test_sft_workspace_size():
    L = radar.lib()
    cfg = radar.Config(1024, 256, 1024, 256, 1024, zc_root=7)
    s = radar.sft_desc(8)
    assert L.radar_fps_sft_workspace_size(ctypes.byref(cfg.desc()), ctypes.byref(s), 3) == _al(3 * 8 * 3 * 1024 * 8)
    s2 = radar.sft_desc(4, dirs=[(1, 1), (3, -5)])
    assert L.radar_fps_sft_workspace_size(ctypes.byref(cfg.desc()), ctypes.byref(s2), 1) == _al(2 * 3 * 1024 * 8)


def test_sft_workspace_size_prime_factor_path():
    # Table I's frame: N = 2048, M = 560, Q = lcm = 71680 = 2048 * 35
    L = radar.lib()
    cfg = radar.Config(2048, 560, 2048, 560, 2048, zc_root=7)
    s = radar.sft_desc(8)
    spectra = _al(8 * 3 * 71680 * 8)
    # the spectra, the first pass's output, conj(z_k) for k < N, W_35^x
    assert L.radar_fps_sft_workspace_size(ctypes.byref(cfg.desc()), ctypes.byref(s), 1) == \
        2 * spectra + _al(2048 * 8) + _al(35 * 8)
    # other sizes of the path are accepted: odd N (the k(k+1) phase of Eq. 23), N not a power of two
    for n, m, root in ((45, 64, 7), (96, 40, 5), (1000, 64, 3), (2048, 560, 1)):
        c = radar.Config(n, m, n, m, n, zc_root=root)
        assert L.radar_fps_sft_workspace_size(ctypes.byref(c.desc()), ctypes.byref(s), 1) > 0, (n, m)


@pytest.mark.parametrize("change,code", [
    (dict(k=0), radar.RADAR_E_ARG), (dict(k=65), radar.RADAR_E_ARG),
    (dict(n_dirs=0), radar.RADAR_E_ARG), (dict(n_dirs=17), radar.RADAR_E_ARG),
    (dict(pfa=0.0), radar.RADAR_E_ARG), (dict(pfa=1.0), radar.RADAR_E_ARG),
    (dict(tol=0.0), radar.RADAR_E_ARG), (dict(flags=1), radar.RADAR_E_ARG),
    (dict(dir0=(0, 0)), radar.RADAR_E_ARG), (dict(dir0=(256, -64)), radar.RADAR_E_ARG),  # both vanish mod (N, M)
    (dict(n_sub=8), radar.RADAR_E_UNSUPPORTED), (dict(n_sym=8192), radar.RADAR_E_UNSUPPORTED),
    (dict(zc_root=4), radar.RADAR_E_NOT_COPRIME),
    # Q = lcm(N, M) not a power of two: the prime-factor path's limits
    (dict(n_sub=45, n_sym=63), radar.RADAR_E_UNSUPPORTED),       # Q = 315: power of two in Q below 16
    (dict(n_sub=272, n_sym=304), radar.RADAR_E_UNSUPPORTED),     # odd part of Q = 17 * 19 > 255
    (dict(n_sub=4096, n_sym=4095), radar.RADAR_E_UNSUPPORTED),   # Q above 131072
    (dict(n_sub=96, zc_root=3), radar.RADAR_E_NOT_COPRIME),      # gcd(3, 96) = 3
    (dict(refine=True), radar.RADAR_E_ARG),
])
def test_sft_validation_rejects(change, code):
    base = dict(n_sub=256, n_sym=64, n_pad=256, m_pad=64, n_cp=256, zc_root=1)
    for key in ("n_sub", "n_sym", "zc_root", "refine"):
        if key in change:
            base[key] = change[key]
    cfg = radar.Config(**base)
    s = radar.sft_desc(4)
    for key in ("k", "n_dirs", "pfa", "tol", "flags"):
        if key in change:
            setattr(s, key, change[key])
    if "dir0" in change:
        s.dirs[0][0], s.dirs[0][1] = change["dir0"]
    L = radar.lib()
    assert L.radar_fps_sft_workspace_size(ctypes.byref(cfg.desc()), ctypes.byref(s), 1) == 0
    # validation happens before any HIP call: dummy non-null pointers are never touched
    p = 256
    assert L.radar_fps_sft(ctypes.byref(cfg.desc()), ctypes.byref(s), 1, p, p, 0, p, p, p, None, p, 1 << 40,
                           None) == code


def test_sft_rejects_pointers_and_workspace():
    L = radar.lib()
    cfg = radar.Config(256, 64, 256, 64, 256, zc_root=1)
    s = radar.sft_desc(4)
    d, sp = ctypes.byref(cfg.desc()), ctypes.byref(s)
    need = L.radar_fps_sft_workspace_size(d, sp, 2)
    p = 256
    assert L.radar_fps_sft(d, sp, 2, p, p, 256 * 64, p, p, p, None, p, need - 1, None) == radar.RADAR_E_WORKSPACE
    assert L.radar_fps_sft(d, sp, 2, p, p, 256 * 64, p, p, p, None, None, need, None) == radar.RADAR_E_ARG
    assert L.radar_fps_sft(d, sp, 2, None, p, 256 * 64, p, p, p, None, p, need, None) == radar.RADAR_E_ARG
    assert L.radar_fps_sft(d, sp, 2, p, p, 100, p, p, p, None, p, need, None) == radar.RADAR_E_ARG  # overlap
    assert L.radar_fps_sft(d, sp, 0, p, p, 0, p, p, p, None, p, need, None) == radar.RADAR_E_ARG


@pytest.mark.parametrize("kw,code", [
    (dict(precision=radar.FLAG_BF16X3 | radar.FLAG_FP16X3), radar.RADAR_E_ARG),   # at most one form
    (dict(precision=8), radar.RADAR_E_ARG),                                        # unknown bit
    (dict(precision=radar.FLAG_BF16X3, n_pad=2048), radar.RADAR_E_UNSUPPORTED),   # needs N' = 4N
    (dict(precision=radar.FLAG_FP16X3, n_cp=300), radar.RADAR_E_UNSUPPORTED),     # needs 4 N_cp <= N
    (dict(precision=radar.FLAG_FP16 | radar.FLAG_FP16X3), radar.RADAR_E_ARG),     # at most one form
    (dict(precision=radar.FLAG_FP16 | radar.FLAG_BF16X3), radar.RADAR_E_ARG),
    (dict(precision=radar.FLAG_FP16, n_sub=512, n_pad=2048, n_cp=128), radar.RADAR_E_UNSUPPORTED),  # N = 1024 only
    (dict(precision=radar.FLAG_FP16, n_pad=8192), radar.RADAR_E_UNSUPPORTED),     # needs N' = 4N
    (dict(precision=radar.FLAG_FP16, n_cp=257), radar.RADAR_E_UNSUPPORTED),       # needs 4 N_cp <= N
])
def test_precision_flag_validation(kw, code):
    base = dict(n_sub=1024, n_sym=1024, n_pad=4096, m_pad=4096, n_cp=256, zc_root=7)
    base.update(kw)
    cfg = radar.Config(**base)
    L = radar.lib()
    assert L.radar_frame_workspace_size(ctypes.byref(cfg.desc()), 1, 8) == 0
    p = 256
    assert L.radar_frame_process(ctypes.byref(cfg.desc()), 1, p, p, 0, p, 0, 8, p, p, p, p, 1 << 40, None) == code


def test_fp16_form_takes_both_outputs():
    # with P written or peaks only (its rows then rescanned in FP32), the FP16
    # form passes validation and stops at the workspace check, before any HIP call
    L = radar.lib()
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7, precision=radar.FLAG_FP16)
    d = ctypes.byref(cfg.desc())
    need = L.radar_frame_workspace_size(d, 1, 8)
    assert need > 0
    p = 256
    assert L.radar_frame_process(d, 1, p, p, 0, None, 0, 8, p, p, p, p, need - 1, None) == radar.RADAR_E_WORKSPACE
    assert L.radar_frame_process(d, 1, p, p, 0, p, 0, 8, p, p, p, p, need - 1, None) == radar.RADAR_E_WORKSPACE


def test_precision_flags_accepted():
    L = radar.lib()
    for fl in (radar.FLAG_BF16X3, radar.FLAG_FP16X3, radar.FLAG_BF16X3 | radar.FLAG_REFINE):
        cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7, precision=fl & ~radar.FLAG_REFINE,
                           refine=bool(fl & radar.FLAG_REFINE))
        assert L.radar_frame_workspace_size(ctypes.byref(cfg.desc()), 1, 8) > 0


def _job(cfg, k, ld=None):
    j = radar.FrameJob()
    j.d = cfg.desc(ld=ld)
    j.Y = j.A = j.P = j.peaks = j.n_peaks = j.status = 256
    j.k = k
    return j


def test_batch_workspace_groups_by_shape():
    L = radar.lib()
    a = radar.Config(256, 64, 1024, 256, 32, zc_root=1)
    b = radar.Config(1024, 256, 4096, 1024, 256, zc_root=7)
    jobs = (radar.FrameJob * 6)(_job(a, 3), _job(b, 8), _job(a, 3), _job(a, 3), _job(b, 8), _job(a, 4))
    ref = 48  # six device pointers per job table entry
    # job tables, then every group's own scratch (groups may run concurrently)
    want = _al(3 * ref) + _al(2 * ref) + _al(1 * ref) + _ws(a, 3, 3) + _ws(b, 2, 8) + _ws(a, 1, 4)
    assert L.radar_batch_workspace_size(jobs, 6) == want
    # a different ld is a different group
    jobs2 = (radar.FrameJob * 2)(_job(a, 3), _job(a, 3, ld=300))
    assert L.radar_batch_workspace_size(jobs2, 2) == 2 * _al(ref) + 2 * _ws(a, 1, 3)


def test_batch_rejects_before_any_hip_call():
    L = radar.lib()
    a = radar.Config(256, 64, 1024, 256, 32, zc_root=1)
    out = ctypes.c_void_p()
    good = (radar.FrameJob * 1)(_job(a, 3))
    assert L.radar_batch_workspace_size(good, 0) == 0
    assert L.radar_batch_create(good, 0, 0, 256, 1 << 30, None, ctypes.byref(out)) == radar.RADAR_E_ARG
    assert L.radar_batch_create(good, 1, 8, 256, 1 << 30, None, ctypes.byref(out)) == radar.RADAR_E_ARG  # flag
    assert L.radar_batch_create(good, 1, 0, 256, 1 << 30, None, None) == radar.RADAR_E_ARG
    bad = (radar.FrameJob * 2)(_job(a, 3), _job(radar.Config(1000, 64, 4000, 256, 32), 3))
    assert L.radar_batch_workspace_size(bad, 2) == 0
    assert L.radar_batch_create(bad, 2, 0, 256, 1 << 30, None, ctypes.byref(out)) == radar.RADAR_E_UNSUPPORTED
    nok = (radar.FrameJob * 1)(_job(a, 65))
    assert L.radar_batch_create(nok, 1, 0, 256, 1 << 30, None, ctypes.byref(out)) == radar.RADAR_E_ARG
    nul = (radar.FrameJob * 1)(_job(a, 3))
    nul[0].P = None
    assert L.radar_batch_create(nul, 1, 0, 256, 1 << 30, None, ctypes.byref(out)) == radar.RADAR_E_ARG
    assert L.radar_batch_launch(None, None) == radar.RADAR_E_ARG
