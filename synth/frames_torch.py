"""Seeded synthetic radar frames built on the GPU, for batches too large to
draw on the host.

Same recipe as synth/frames.py (QAM symbols, the transmitter's ZC precoding,
point targets with Rayleigh amplitudes, circular AWGN): the target parameters
are drawn on the host by frames.draw_targets from the same seed sequence, and
the M x N arrays are formed on the device with torch.  Holds no receiver
arithmetic.
"""

from __future__ import annotations

import functools
import math

import numpy as np
import torch

from synth import frames as S


@functools.lru_cache(maxsize=4)
def _dense_matrix(n: int, root: int, shift: int) -> np.ndarray:
    # the transmitter's N x N matrix Z[i, j] = zc(i N + j) of a length-N^2 sequence
    return S.tx_precoding_sequence(n * n, root, shift).reshape(n, n)


def make_frame(spec: S.FrameSpec, config_id: int, frame_index: int, device="cuda"):
    """One frame on `device`: (Y, A) complex64 (M, N) plus the targets (rho, nu, b)."""
    rng = S.rng_for(config_id, frame_index)
    rho, nu, b = S.draw_targets(rng, spec)
    n, m = spec.n_sub, spec.n_sym
    g = torch.Generator(device=device)
    g.manual_seed(int(rng.integers(0, 2 ** 62)))
    if spec.qam == 4:
        lv, norm = torch.tensor([-1.0, 1.0], device=device), math.sqrt(2.0)
    else:
        lv, norm = torch.tensor([-3.0, -1.0, 1.0, 3.0], device=device), math.sqrt(10.0)
    re = lv[torch.randint(0, lv.numel(), (m, n), generator=g, device=device)]
    im = lv[torch.randint(0, lv.numel(), (m, n), generator=g, device=device)]
    A = torch.complex(re, im) / norm
    k = torch.arange(n, dtype=torch.float64, device=device)
    l = torch.arange(m, dtype=torch.float64, device=device)
    echo = torch.zeros((m, n), dtype=torch.complex128, device=device)
    for p in range(spec.n_targets):
        dop = torch.exp(2j * math.pi * l * float(nu[p]) / m)
        rng_ph = torch.exp(-2j * math.pi * k * float(rho[p]) / n)
        echo += complex(b[p]) * torch.outer(dop, rng_ph)
    tx = A.to(torch.complex128)
    if spec.zc_root is not None and spec.zc_dense:
        Z = torch.from_numpy(_dense_matrix(n, spec.zc_root, spec.zc_shift)).to(device)
        tx = (tx @ Z.transpose(0, 1).contiguous()) / math.sqrt(n)
    elif spec.zc_root is not None:
        z = torch.from_numpy(S.tx_precoding_sequence(n, spec.zc_root, spec.zc_shift)).to(device)
        tx = tx * z[None, :]
    Y = tx * echo
    if spec.noise:
        sigma2 = 10.0 ** (-spec.snr_db / 10.0)
        w = torch.complex(torch.randn((m, n), generator=g, device=device, dtype=torch.float64),
                          torch.randn((m, n), generator=g, device=device, dtype=torch.float64))
        Y = Y + w * math.sqrt(sigma2 / 2.0)
    return Y.to(torch.complex64), A.to(torch.complex64), (np.asarray(rho), np.asarray(nu), np.asarray(b))


def monte_carlo_specs(n_frames: int, seed: int = 3):
    """The uneven Monte-Carlo workload: N in {256, 512, 1024, 2048}, M in
    {64, ..., 1024}, SNR uniform in [-20, 10] dB, 1-16 off-grid Rayleigh
    targets inside the DFT-CE range box (N_cp = N/4), 16-QAM, ZC root 7."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(n_frames):
        n = int(rng.choice([256, 512, 1024, 2048]))
        m = int(rng.choice([64, 128, 256, 512, 1024]))
        specs.append(S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=7, n_targets=int(rng.integers(1, 17)),
                                 snr_db=float(rng.uniform(-20.0, 10.0)), on_grid=False, rho_min=1.0,
                                 rho_max=n / 4 - 1.0, nu_abs_max=m / 2 - 1.0, rayleigh=True, min_sep=3.0))
    return specs
