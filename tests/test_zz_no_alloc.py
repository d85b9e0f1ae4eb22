"""radar_frame_process_noalloc (the entry point for callers that cannot
allocate) against radar_frame_process with a caller workspace, through the C
ABI: the same kernels on the same inputs, so every output must be identical.
Two calls in a row share the library's one workspace array; the second is
smaller, so it runs on what the first left behind."""

import numpy as np
import pytest

from synth import frames as S
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
radar = pytest.importorskip("paper_2209_03883_amd.radar")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    radar.lib()  # fail loudly if the HIP library is missing


def _both(Yd, Ad, cfg, k, materialise=True):
    F = Yd.shape[0]
    dev = Yd.device
    P0, pk0, n0, st0 = radar.frame_process(Yd, Ad, cfg, k, materialise=materialise)
    P1 = torch.full((F, cfg.m_pad, cfg.n_pad), float("nan"), device=dev) if materialise else None
    pk1 = torch.full((F, k, radar.PEAK_WORDS), -7, dtype=torch.int32, device=dev)
    n1 = torch.full((F,), -7, dtype=torch.int32, device=dev)
    st1 = torch.full((F,), -7, dtype=torch.int32, device=dev)
    radar.frame_process_noalloc(Yd, Ad, cfg, k, P=P1, peaks=pk1, n_peaks=n1, status=st1)
    torch.cuda.synchronize()
    if materialise:
        assert torch.equal(P0, P1), "periodograms differ"
    assert torch.equal(n0, n1), (n0.cpu(), n1.cpu())
    assert torch.equal(st0, st1), (st0.cpu(), st1.cpu())
    for f in range(F):
        n = int(n0[f])
        assert torch.equal(pk0[f, :n], pk1[f, :n]), f"frame {f}: peaks differ"
    return n0


def test_noalloc_two_calls_second_smaller():
    # call 1: two full 1024 x 1024 frames (about 20.6 MiB of workspace)
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7, window=radar.WIN_HANN)
    frames = [S.make_frame(S.spec_full(snr_db=0.0), 2, i) for i in range(2)]
    Y, A = S.frames_to_complex64(frames)
    say("no-alloc call 1: two 1024x1024 frames, k = 8")
    n = _both(torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda(), cfg, 8)
    assert bool((n == 8).all().cpu())
    # call 2: three small frames on the same array, rows and counts of call 1 still in it
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1, window=radar.WIN_HANN)
    frames = [S.make_frame(S.spec_small(snr_db=0.0), 1, i) for i in range(3)]
    Y, A = S.frames_to_complex64(frames)
    say("no-alloc call 2: three 256x64 frames, k = 3")
    n = _both(torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda(), cfg, 3)
    assert bool((n == 3).all().cpu())
    # call 3: peaks only (P not written) with threshold detection and refinement
    cfg = radar.Config(256, 64, 1024, 256, 32, zc_root=1, window=radar.WIN_HANN, refine=True, threshold=True,
                       pfa=1e-3, noise_power=1.0)
    say("no-alloc call 3: peaks only, threshold and refinement")
    _both(torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda(), cfg, 8, materialise=False)
    # call 4: a full frame in the FP16 form, peaks only (its rows rescanned in FP32)
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7, window=radar.WIN_HANN, precision=radar.FLAG_FP16)
    frames = [S.make_frame(S.spec_full(snr_db=0.0), 2, 5)]
    Y, A = S.frames_to_complex64(frames)
    say("no-alloc call 4: FP16 form, peaks only, one 1024x1024 frame")
    n = _both(torch.from_numpy(Y).cuda(), torch.from_numpy(A).cuda(), cfg, 8, materialise=False)
    assert bool((n == 8).all().cpu())


def test_noalloc_rejects_beyond_its_workspace():
    cfg = radar.Config(1024, 1024, 4096, 4096, 256, zc_root=7, window=radar.WIN_HANN)
    need = radar.workspace_bytes(cfg, 4, 8)
    assert need > 32 << 20
    Y = torch.zeros((4, 1024, 1024), dtype=torch.complex64, device="cuda")
    P = torch.empty((4, 4096, 4096), dtype=torch.float32, device="cuda")
    pk = radar.alloc_peaks(4, 8, "cuda")
    n = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(radar.RadarError) as e:
        radar.frame_process_noalloc(Y, Y, cfg, 8, P=P, peaks=pk, n_peaks=n, status=st)
    assert e.value.code == radar.RADAR_E_WORKSPACE
    del P
    torch.cuda.synchronize()
