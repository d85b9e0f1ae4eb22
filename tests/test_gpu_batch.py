"""Batches of frames with uneven shapes (radar_batch_*) through the C ABI:
every job's periodogram and peaks against the same frame processed alone by
radar_frame_process, and the first job of every shape group against the FP64
oracle; graph replays are checked one by one with eager work between them."""

import numpy as np
import pytest

from oracle import radar_oracle as O
from synth import frames as S
from tests.gpu_util import P_TOL_FP32, compare_peak_indices, normwise_error, oracle_ranked, rounded, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
radar = pytest.importorskip("paper_2209_03883_amd.radar")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    radar.lib()


# (N, M, N', M', N_cp, window, zc root, k, flags, ld)
SHAPES = [
    (256, 64, 1024, 256, 32, radar.WIN_HANN, 1, 3, 0, None),
    (512, 128, 2048, 512, 128, radar.WIN_HAMMING, 3, 5, 0, None),
    (1024, 256, 4096, 1024, 256, radar.WIN_HANN, 7, 8, radar.FLAG_REFINE, None),
    (2048, 64, 8192, 256, 512, radar.WIN_HANN, 7, 8, 0, None),
    (128, 32, 256, 64, 16, radar.WIN_RECT, 5, 4, 0, None),          # generic range kernel
    (1024, 128, 4096, 512, 256, radar.WIN_HANN, 7, 8, radar.FLAG_BF16X3, None),
    (256, 64, 1024, 256, 32, radar.WIN_HANN, 1, 3, 0, 320),         # strided rows
]
# frames per shape (uneven), in an interleaved order
ORDER = [0, 1, 2, 0, 3, 4, 5, 0, 1, 6, 2, 4, 6, 0]


def _frame(shape, i):
    n, m, nq, mp, ncp, win, root, k, flags, ld = shape
    spec = S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=root, n_targets=1 + (i * 5) % 16,
                       snr_db=-20.0 + (i * 7.3) % 30.0, on_grid=False, rho_min=1.0, rho_max=ncp - 1.0,
                       nu_abs_max=m / 2 - 1, rayleigh=True, min_sep=1.0)
    return S.make_frame(spec, 30, i)


def _cfg(shape):
    n, m, nq, mp, ncp, win, root, k, flags, ld = shape
    return radar.Config(n, m, nq, mp, ncp, zc_root=root, window=win, refine=bool(flags & radar.FLAG_REFINE),
                        precision=flags & ~radar.FLAG_REFINE)


def _device(frame, ld):
    Y = torch.from_numpy(frame.Y.astype(np.complex64)).cuda()
    A = torch.from_numpy(frame.A.astype(np.complex64)).cuda()
    if ld is not None:
        Yp = torch.zeros((Y.shape[0], ld), dtype=torch.complex64, device="cuda")
        Ap = torch.ones((A.shape[0], ld), dtype=torch.complex64, device="cuda")
        Yp[:, :Y.shape[1]] = Y
        Ap[:, :A.shape[1]] = A
        Y, A = Yp[:, :Y.shape[1]], Ap[:, :A.shape[1]]
    return Y, A


def _setup():
    jobs, frames = [], []
    for i, si in enumerate(ORDER):
        shape = SHAPES[si]
        f = _frame(shape, i)
        Y, A = _device(f, shape[9])
        jobs.append((Y, A, _cfg(shape), shape[7]))
        frames.append((f, shape))
    return jobs, frames


def _alone(job):
    Y, A, cfg, k = job
    P, pk, n_pk, st = radar.frame_process(Y, A, cfg, k)
    torch.cuda.synchronize()
    return P[0].cpu().numpy(), radar.unpack_peaks(pk, n_pk.cpu())[0], int(st.cpu()[0])


def _clobber(b):
    for P, pk, npk, st in zip(b.P, b.peaks, b.n_peaks, b.status):
        P.fill_(float("nan"))
        pk.fill_(-1)
        npk.fill_(-1)
        st.fill_(-1)


@pytest.mark.parametrize("graph", [True, False])
def test_batch_matches_frames_alone(graph):
    jobs, frames = _setup()
    say(f"batch of {len(jobs)} uneven jobs, graph={graph}")
    alone = [_alone(j) for j in jobs]
    b = radar.Batch(jobs, graph=graph)
    assert len(b.groups()) == len(SHAPES)
    for rep in range(3):
        _clobber(b)
        b.launch()
        torch.cuda.synchronize()
        for i in range(len(jobs)):
            P, pk, st = b.results(i)
            Pa, pka, sta = alone[i]
            assert st == sta == 0, (rep, i)
            np.testing.assert_array_equal(P, Pa)
            assert pk == pka, (rep, i)
        # eager work between replays
        _alone(jobs[rep])
        say(f"replay {rep}: {len(jobs)} jobs identical to frames processed alone")
    b.close()


def test_batch_first_job_of_every_group_matches_oracle():
    """The first job of every shape group against the FP64 oracle, flagged
    groups included: the periodogram at the form's tolerance (1e-5 for FP32,
    2e-3 for the BF16x3 matrix-core range stage), the peak cells up to
    near-ties, and the refinement group's sub-cell positions within 2e-4 cells
    of the oracle's refine_peak."""
    jobs, frames = _setup()
    b = radar.Batch(jobs, graph=True)
    b.launch()
    torch.cuda.synchronize()
    seen = set()
    for i, (f, shape) in enumerate(frames):
        si = SHAPES.index(shape)
        if si in seen:
            continue
        seen.add(si)
        n, m, nq, mp, ncp, win, root, k, flags, ld = shape
        P, pk, st = b.results(i)
        assert st == 0
        P_ref = O.frame_periodogram(rounded(f.Y), rounded(f.A), n_pad=nq, m_pad=mp, n_cp=ncp, window_kind=win,
                                    zc_root=root)
        err = normwise_error(P, P_ref)
        tol = 2e-3 if flags & radar.FLAG_BF16X3 else P_TOL_FP32
        assert err <= tol, (i, shape, err)
        ref = oracle_ranked(O, P_ref, k)
        excl = compare_peak_indices([(s, r) for s, r, *_ in pk], ref, P_ref,
                                    near_tie=1e-3 if flags & radar.FLAG_BF16X3 else 1e-5)
        assert excl is not None and excl <= 1, (i, shape, pk[:3], ref[:3])
        line = f"group {si} ({n}x{m}, flags {flags}) job {i}: normwise P error {err:.2e}"
        if flags & radar.FLAG_REFINE:
            Hw = O.windowed_estimate(rounded(f.Y), rounded(f.A), n_cp=ncp, window_kind=win, zc_root=root)
            worst = 0.0
            for (gs, gr, _, gso, gro), (rs, rr, rv) in zip(pk, ref):
                if (gs, gr) != (rs, rr):
                    continue  # a near-tie: another cell, another refinement
                so, ro = O.refine_peak(Hw, rs, rr, nq, mp)
                worst = max(worst, abs(gso - so), abs(gro - ro))
            assert worst <= 2e-4, (i, worst)
            line += f", refined positions within {worst:.1e} cells"
        say(line)
    assert len(seen) == len(SHAPES)
    b.close()


def test_batch_autotuned_plan():
    jobs, frames = _setup()
    alone = [_alone(j) for j in jobs]
    b = radar.Batch(jobs, graph=True, tune=True)
    plans = b.plans()
    say(f"tuned plans: {plans}")
    for pl in plans:
        assert pl["k1_mult"] in (1, 2) and pl["k3_mult"] in (1, 2) and pl["k3_generic"] in (0, 1)
        assert pl["k2_half_tile"] in (0, 1) and pl["scan_groups"] in (32, 128)
    for rep in range(2):
        _clobber(b)
        b.launch()
        torch.cuda.synchronize()
        for i in range(len(jobs)):
            P, pk, st = b.results(i)
            Pa, pka, _ = alone[i]
            assert st == 0
            # a tuned plan may pick another range kernel: same values up to FP32 rounding
            assert normwise_error(P, Pa) <= 1e-5, i
            assert compare_peak_indices([(s, r) for s, r, *_ in pk], [(s, r, Pa[s + P.shape[0] // 2, r])
                                                                      for s, r, *_ in pka], Pa) is not None
    b.close()
