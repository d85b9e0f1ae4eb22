"""GPU parity of the sub-cell peak refinement (RADAR_FLAG_REFINE of
radar_frame_process) against the FP64 oracle's refine_peak, through the C ABI."""

import numpy as np
import pytest

from oracle import radar_oracle as O
from synth import frames as S
from tests.gpu_util import compare_peak_indices, oracle_ranked, rounded, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
radar = pytest.importorskip("paper_2209_03883_amd.radar")

# Refined positions (grid cell + offset) agree with the oracle within this many
# cells of the N' x M' grid.  The fit turns a relative error e of P on the fine
# cells into a position error of about e / c fine cells, where c (>= 0.004 per
# fine cell^2 for the Hann and Hamming main lobes) is the curvature of ln P.
# With e ~ 1e-6 (FP32 Doppler sums of FP32 taps at a target peak) that is
# ~2.5e-4 fine cells; the largest difference seen on the full 1024 x 1024 frame
# is 1.3e-5 cells.
POS_TOL = 2e-4


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    radar.lib()


def _run(Y, A, cfg, k):
    Yd = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.complex64)).cuda()
    Ad = torch.from_numpy(np.ascontiguousarray(A, dtype=np.complex64)).cuda()
    P, peaks, n_peaks, status = radar.frame_process(Yd, Ad, cfg, k)
    torch.cuda.synchronize()
    return P.cpu().numpy(), radar.unpack_peaks(peaks, n_peaks.cpu()), status.cpu().numpy()


def _oracle(Y, A, cfg, k):
    Y, A = rounded(Y), rounded(A)
    P = O.frame_periodogram(Y, A, n_pad=cfg.n_pad, m_pad=cfg.m_pad, n_cp=cfg.n_cp, window_kind=cfg.window,
                            zc_root=cfg.zc_root, zc_shift=cfg.zc_shift)
    Hw = O.windowed_estimate(Y, A, n_cp=cfg.n_cp, window_kind=cfg.window, zc_root=cfg.zc_root,
                             zc_shift=cfg.zc_shift)
    ref = oracle_ranked(O, P, k)
    offs = [O.refine_peak(Hw, s, r, cfg.n_pad, cfg.m_pad) for s, r, _ in ref]
    return P, ref, offs


def _check(Y, A, cfg, k, label, min_rel=0.0):
    P_gpu, pk, st = _run(Y[None], A[None], cfg, k)
    assert st[0] == 0
    P_ref, ref, offs = _oracle(Y, A, cfg, k)
    assert compare_peak_indices([(s, r) for s, r, *_ in pk[0]], ref, P_ref) is not None, label
    pmax = ref[0][2]
    worst = 0.0
    checked = 0
    for (gs, gr, _, gso, gro), (rs, rr, rv), (so, ro) in zip(pk[0], ref, offs):
        if (gs, gr) != (rs, rr) or rv < min_rel * pmax:
            continue
        d = max(abs((gs + gso) - (rs + so)), abs((gr + gro) - (rr + ro)))
        worst = max(worst, d)
        checked += 1
        assert d <= POS_TOL, (label, (gs, gr, gso, gro), (rs, rr, so, ro), d)
    say(f"{label}: {checked} refined peaks, worst position difference {worst:.2e} cells")
    assert checked > 0
    return pk[0], ref, offs


@pytest.mark.parametrize("frame_index", [0, 1])
def test_refine_small_workload(frame_index):
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1, window=radar.WIN_HANN, refine=True)
    f = S.make_frame(S.spec_small(snr_db=0.0), 1, frame_index)
    say(f"refine small workload frame {frame_index}")
    pk, _, _ = _check(f.Y, f.A, cfg, 3, f"refine-small/{frame_index}")
    # on-grid targets: the refined positions sit on the native bins
    for s, r, _, so, ro in pk:
        assert abs(s + so - round(s + so)) < 0.05 and abs(r + ro - round(r + ro)) < 0.05


@pytest.mark.parametrize("snr_db", [0.0, 10.0])
def test_refine_full_frame(snr_db):
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7, window=radar.WIN_HANN, refine=True)
    f = S.make_frame(S.spec_full(snr_db=snr_db), 2, 40 + int(snr_db))
    say(f"refine full frame snr {snr_db}")
    _check(f.Y, f.A, cfg, 8, f"refine-full/{snr_db}")


@pytest.mark.parametrize("shape", [
    (64, 32, 256, 512, 64, radar.WIN_HAMMING),   # 16x Doppler padding: one fine cell per cell
    (128, 64, 128, 128, 32, radar.WIN_HANN),     # no padding: 16 fine cells per cell
    (512, 128, 4096, 512, 512, radar.WIN_HANN),  # 8x range padding, N_cp = N (two range chunks)
])
def test_refine_shapes(shape):
    n, m, nq, mp, ncp, win = shape
    spec = S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=3, n_targets=2, snr_db=5.0, on_grid=False,
                       rho_min=1.0, rho_max=min(ncp, n) - 2.0, nu_abs_max=m / 2 - 2.0, min_sep=6.0)
    f = S.make_frame(spec, 93, n + m)
    cfg = radar.Config(n, m, nq, mp, ncp, zc_root=3, window=win, refine=True)
    say(f"refine shape {shape}")
    _check(f.Y, f.A, cfg, 2, f"refine-shape/{shape}", min_rel=1e-2)


def test_refine_noiseless_targets_land_on_truth():
    n, m, nq, mp = 512, 128, 2048, 512
    spec = S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=5, n_targets=2, noise=False, on_grid=False,
                       rho_min=20.0, rho_max=200.0, nu_abs_max=50.0, min_sep=40.0)
    f = S.make_frame(spec, 94, 0)
    cfg = radar.Config(n, m, nq, mp, n, zc_root=5, window=radar.WIN_HANN, refine=True)
    say("refine noiseless targets")
    _, pk, _ = _run(f.Y[None], f.A[None], cfg, 2)
    got = sorted(((s + so) * m / mp, (r + ro) * n / nq) for s, r, _, so, ro in pk[0])
    want = sorted(zip(f.nu, f.rho))
    for (gv, gr), (tv, tr) in zip(got, want):
        assert abs(gv - tv) < 3e-3 and abs(gr - tr) < 3e-3, (got, want)


def test_refine_leaves_periodogram_and_cells_unchanged():
    base = dict(n_sub=256, n_sym=64, n_pad=1024, m_pad=256, n_cp=32, zc_root=1)
    f = S.make_frame(S.spec_small(snr_db=0.0), 1, 5)
    say("refine on/off")
    P0, pk0, _ = _run(f.Y[None], f.A[None], radar.Config(**base), 3)
    P1, pk1, _ = _run(f.Y[None], f.A[None], radar.Config(**base, refine=True), 3)
    np.testing.assert_array_equal(P0, P1)
    assert [p[:3] for p in pk0[0]] == [p[:3] for p in pk1[0]]
    assert all(p[3] == 0.0 and p[4] == 0.0 for p in pk0[0])
