"""GPU parity of the time-domain frame simulation (radar_simulate_frames,
Sec. II-B.1 Eq. 1-2 and 7-10) against the FP64 oracle, and what it shows
about Eq. 11's frequency-domain model.

The oracle evaluates the OFDM waveform sample by sample from its definition;
the GPU forms each symbol with one inverse FFT per target and one forward
FFT.  Tolerance: max |Y_gpu - Y_ref| <= 2e-6 max |Y_ref| (FP32 transforms of
a few unit-amplitude terms; phases reduced to [0, 1) cycles before the FP32
sincos).
"""

import numpy as np
import pytest

from oracle import radar_oracle as O
from synth import frames as S
from tests.gpu_util import rounded, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
radar = pytest.importorskip("paper_2209_03883_amd.radar")

TOL = 2e-6


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    radar.lib()


def _symbols(rng, F, m, n):
    return ((rng.choice([-3.0, -1.0, 1.0, 3.0], (F, m, n)) + 1j * rng.choice([-3.0, -1.0, 1.0, 3.0], (F, m, n)))
            / np.sqrt(10.0)).astype(np.complex64)


def _run(A, tg, n_guard, fc_df, noise=None):
    F = A.shape[0]
    targets = torch.zeros((F, max(len(t) for t in tg), 4), dtype=torch.float32)
    for f, lst in enumerate(tg):
        for p, (rho, nu, b) in enumerate(lst):
            targets[f, p] = torch.tensor([rho, nu, b.real, b.imag])
    nt = torch.tensor([len(t) for t in tg], dtype=torch.int32)
    Y, st = radar.simulate_frames(torch.from_numpy(A).cuda(), targets.cuda(), nt.cuda(), n_guard=n_guard,
                                  fc_over_df=fc_df, noise=None if noise is None else torch.from_numpy(noise).cuda())
    torch.cuda.synchronize()
    return Y.cpu().numpy(), st.cpu().numpy()


def _ref(A, tg, n_guard, fc_df, noise=None):
    # the oracle sees the FP32 values the GPU sees
    return O.simulate_frame(rounded(A), [(float(np.float32(r)), float(np.float32(v)), complex(np.complex64(b)))
                                         for r, v, b in tg], n_guard=n_guard, fc_over_df=fc_df,
                            noise=None if noise is None else rounded(noise))


# (N, M, n_guard): the one-thread teams, single-wave teams and multi-wave teams
SIM_SHAPES = [(16, 16, 4), (64, 16, 16), (256, 32, 64), (2048, 16, 512)]


@pytest.mark.parametrize("shape", SIM_SHAPES, ids=[f"{s[0]}x{s[1]}-g{s[2]}" for s in SIM_SHAPES])
@pytest.mark.parametrize("fc_df", [77e9 / 240e3, 40.0])
def test_simulation_matches_oracle(shape, fc_df):
    n, m, ng = shape
    rng = np.random.default_rng(n + int(fc_df))
    A = _symbols(rng, 2, m, n)
    tg = []
    for f in range(2):
        lst = []
        for p in range(3):
            nu = float(rng.uniform(-(m / 2 - 1), m / 2 - 1))
            # a delay that stays inside the prefix while the target migrates
            drift = nu * n / (m * (n + ng)) / fc_df * ((m - 1) * (n + ng) + ng)
            lo, hi = max(0.0, -drift), ng - max(0.0, drift)
            if hi <= lo:
                nu, lo, hi = 0.0, 0.0, float(ng)
            rho = float(rng.uniform(lo, lo + 0.9 * (hi - lo)))
            b = complex(rng.standard_normal() + 1j * rng.standard_normal()) / np.sqrt(2.0)
            lst.append((rho, nu, b))
        tg.append(lst[: 3 - f])  # the frames carry different numbers of targets
    noise = (0.1 * (rng.standard_normal((2, m, n)) + 1j * rng.standard_normal((2, m, n)))).astype(np.complex64)
    say(f"simulation {shape}, fc/df {fc_df:g}")
    Y, st = _run(A, tg, ng, fc_df, noise)
    for f in range(2):
        assert st[f] == 0
        ref = _ref(A[f], tg[f], ng, fc_df, noise[f])
        err = float(np.max(np.abs(Y[f] - ref)) / np.max(np.abs(ref)))
        say(f"frame {f}: max error {err:.2e} of max |Y|")
        assert err <= TOL


def test_simulation_static_targets_equal_eq11():
    # no motion: Eq. 11 exactly (up to FP32)
    rng = np.random.default_rng(5)
    n, m, ng = 256, 16, 64
    A = _symbols(rng, 1, m, n)
    tg = [[(7.0, 0.0, 1.0 + 0j), (30.0, 0.0, 0.5j)]]
    Y, _ = _run(A, tg, ng, 77e9 / 240e3)
    k = np.arange(n)
    eq11 = A[0].astype(np.complex128) * (np.exp(-2j * np.pi * k * 7.0 / n) + 0.5j * np.exp(-2j * np.pi * k * 30.0 / n))
    assert float(np.max(np.abs(Y[0] - eq11))) <= 1e-5


def test_simulation_flags_intersymbol_interference():
    rng = np.random.default_rng(6)
    A = _symbols(rng, 2, 16, 64)
    # frame 1: delay beyond the prefix
    Y, st = _run(A, [[(3.0, 1.0, 1.0 + 0j)], [(20.0, 1.0, 1.0 + 0j)]], 16, 77e9 / 240e3)
    assert st[0] == 0 and st[1] & radar.ST_ISI


def test_ici_and_detection_against_eq11():
    """Full 1024 x 1024 frames, eight off-grid Rayleigh targets spread over
    the whole Doppler range (CFO up to 0.4 subcarrier spacings at the
    unambiguous limit), -20 dB per element.  The time-domain frames differ from
    the Eq. 11 frames by the inter-carrier interference; the receive path finds
    the targets in both."""
    from synth import frames_torch as G

    n = m = 1024
    ng = 256
    spec = S.spec_full(snr_db=-20.0)
    hits = {"eq11": 0, "time": 0}
    tot = 0
    ici = []
    cfg = radar.Config(n, m, 4 * n, 4 * m, ng, zc_root=None, window=radar.WIN_HANN)
    for i in range(4):
        # Eq. 11 frame from the generator (no precoding), and the same symbols,
        # targets and noise through the time-domain model
        sp = S.FrameSpec(**{**spec.__dict__, "zc_root": None})
        Y11, A, (rho, nu, b) = G.make_frame(sp, 66, i)
        k = torch.arange(n, device="cuda", dtype=torch.float64)
        l = torch.arange(m, device="cuda", dtype=torch.float64)
        clean = torch.zeros((m, n), dtype=torch.complex128, device="cuda")   # Eq. 11 channel
        shifted = torch.zeros((m, n), dtype=torch.complex128, device="cuda")  # with the prefix's phase
        for p in range(len(rho)):
            term = complex(b[p]) * torch.outer(torch.exp(2j * np.pi * l * float(nu[p]) / m),
                                               torch.exp(-2j * np.pi * k * float(rho[p]) / n))
            clean += term
            shifted += term * np.exp(2j * np.pi * float(nu[p]) * ng / (m * (n + ng)))
        noise = (Y11.to(torch.complex128) - A.to(torch.complex128) * clean).to(torch.complex64)
        targets = torch.tensor([[float(rho[p]), float(nu[p]), float(b[p].real), float(b[p].imag)]
                                for p in range(len(rho))], dtype=torch.float32, device="cuda")[None]
        nt = torch.tensor([len(rho)], dtype=torch.int32, device="cuda")
        Yt, st = radar.simulate_frames(A[None].contiguous(), targets, nt, n_guard=ng, noise=noise[None].contiguous())
        assert int(st.cpu()[0]) == 0
        # without time scaling (fc/df -> infinity): the ICI alone
        Yi, _ = radar.simulate_frames(A[None].contiguous(), targets, nt, n_guard=ng, fc_over_df=1e30,
                                      noise=noise[None].contiguous())
        # the constant phase of the prefix aside, the difference is what Eq. 11
        # drops: the ICI, and with it the range migration
        sig = A.to(torch.complex128) * shifted
        for Yx, key in ((Yi, "ici"), (Yt, "all")):
            d = Yx[0].to(torch.complex128) - noise.to(torch.complex128) - sig
            ici.append((key, float((d.abs() ** 2).sum() / (sig.abs() ** 2).sum())))
        for key, Y in (("eq11", Y11[None]), ("time", Yt)):
            _, peaks, n_peaks, _ = radar.frame_process(Y.contiguous(), A[None].contiguous(), cfg, 8)
            pk = radar.unpack_peaks(peaks, n_peaks.cpu())[0]
            for r0, v0 in zip(rho, nu):
                for s, r, *_ in pk:
                    ds = (s - v0 * 4 + 2 * m) % (4 * m) - 2 * m
                    if abs(r - r0 * 4) <= 4 and abs(ds) <= 4:
                        hits[key] += 1
                        break
        tot += len(rho)
    say(f"time-domain vs Eq. 11: relative difference energy per frame {[(k, round(x, 3)) for k, x in ici]}; "
        f"targets found (within one native bin) eq11 {hits['eq11']}/{tot}, time-domain {hits['time']}/{tot}")
    assert hits["eq11"] >= tot - 2 and hits["time"] >= tot // 2
