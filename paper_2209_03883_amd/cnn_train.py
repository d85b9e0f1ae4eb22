"""Training data, training loop and evaluation of the CNN sub-cell refiner.

Training frames come from the simulator (synth.frames_torch) and run through
the library's own receive path on the GPU: radar_frame_process (with the
interpolation refinement, the fallback the network is judged against),
radar_cnn_patches, and radar_cnn_train_step.  A patch is labelled with the
offset, in cells of the N' x M' grid, from its detected cell to the true
target position nearest to it; a detection farther than two native bins from
every target is dropped and counted.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from synth import frames as S
from synth import frames_torch as G

from . import radar


@dataclass
class PatchSet:
    patches: torch.Tensor      # (n, 32, 32) float32, device
    labels: torch.Tensor       # (n, 2) float32, device: (range, Doppler) cell offsets
    interp: np.ndarray         # (n, 2) the interpolation refinement's (range, Doppler) offsets
    snr_db: np.ndarray         # (n,)
    dropped: int               # detections with no target within two native bins


def make_patches(n_frames: int, config_id: int, *, n: int = 256, m: int = 64, k: int = 8,
                 snr_db=(-20.0, 10.0), targets=(1, 8), chunk: int = 64, device="cuda") -> PatchSet:
    """Patches and labels from n_frames simulated frames of N = n x M = m,
    4x padding in both axes, N_cp = N/4, Hann, 16-QAM, ZC root 7."""
    rng = np.random.default_rng(np.random.SeedSequence([220903883, 7, config_id]))
    cfg = radar.Config(n, m, 4 * n, 4 * m, n // 4, zc_root=7, window=radar.WIN_HANN, refine=True)
    pats, labs, interp, snrs = [], [], [], []
    dropped = 0
    for c0 in range(0, n_frames, chunk):
        specs = [S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=7, n_targets=int(rng.integers(targets[0], targets[1] + 1)),
                             snr_db=float(rng.uniform(*snr_db)), on_grid=False, rho_min=1.0, rho_max=n / 4 - 1.0,
                             nu_abs_max=m / 2 - 1.0, rayleigh=True, min_sep=3.0)
                 for _ in range(min(chunk, n_frames - c0))]
        frames = [G.make_frame(sp, config_id, c0 + i, device=device) for i, sp in enumerate(specs)]
        Y = torch.stack([f[0] for f in frames])
        A = torch.stack([f[1] for f in frames])
        P, peaks, n_peaks, _ = radar.frame_process(Y, A, cfg, k)
        patches, valid = radar.cnn_patches(P, peaks, n_peaks)
        pk = radar.unpack_peaks(peaks, n_peaks.cpu())
        keep = []
        for f, sp in enumerate(specs):
            rho, nu = frames[f][2][0], frames[f][2][1]
            for i, (s, r, _, so, ro) in enumerate(pk[f]):
                # detection in native bins, distance to each target (Doppler wraps)
                dr = rho - r * n / (4 * n)
                dv = (nu - s * m / (4 * m) + m / 2) % m - m / 2
                j = int(np.argmin(np.hypot(dr, dv)))
                if math.hypot(dr[j], dv[j]) > 2.0:
                    dropped += 1
                    continue
                keep.append(f * k + i)
                labs.append((dr[j] * 4, dv[j] * 4))
                interp.append((ro, so))
                snrs.append(sp.snr_db)
        idx = torch.tensor(keep, dtype=torch.long, device=patches.device)
        pats.append(patches.index_select(0, idx))
        del P, peaks, patches
    return PatchSet(torch.cat(pats).contiguous(), torch.tensor(labs, dtype=torch.float32, device=device),
                    np.asarray(interp, dtype=np.float64), np.asarray(snrs), dropped)


def train(theta0: np.ndarray, data: PatchSet, steps: int, *, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          device="cuda"):
    """Adam on the mean squared error, `steps` steps of `batch` patches (the
    set reshuffled at every pass).  Returns (theta, per-step losses)."""
    theta = torch.from_numpy(np.asarray(theta0, dtype=np.float32)).to(device)
    mom = torch.zeros_like(theta)
    vel = torch.zeros_like(theta)
    ws = radar.CnnWorkspace(batch, True, device)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    n = data.patches.shape[0]
    losses = torch.empty(steps, dtype=torch.float32, device=device)
    order = None
    for t in range(steps):
        j0 = (t * batch) % n
        if order is None or j0 + batch > n:
            order = torch.randperm(n, generator=g, device=device)
            xp = data.patches.index_select(0, order).contiguous()
            yl = data.labels.index_select(0, order).contiguous()
            j0 = 0
        radar.cnn_train_step(theta, mom, vel, t + 1, lr, xp[j0:j0 + batch], yl[j0:j0 + batch], losses[t:t + 1],
                             workspace=ws)
    return theta, losses.cpu().numpy()


def predict(theta: torch.Tensor, patches: torch.Tensor, batch: int = 8192) -> torch.Tensor:
    ws = radar.CnnWorkspace(min(batch, patches.shape[0]), False, patches.device)
    outs = [radar.cnn_forward(theta, patches[i:i + batch].contiguous(), workspace=ws)
            for i in range(0, patches.shape[0], batch)]
    return torch.cat(outs)


def rmse_report(theta: torch.Tensor, data: PatchSet) -> dict:
    """RMSE (cells) of the grid cell alone, the interpolation refinement and
    the network, each axis, over all patches."""
    lab = data.labels.cpu().numpy().astype(np.float64)
    pred = predict(theta, data.patches).cpu().numpy().astype(np.float64)

    def rm(e):
        return [float(np.sqrt(np.mean(e[:, 0] ** 2))), float(np.sqrt(np.mean(e[:, 1] ** 2)))]

    return {"patches": int(lab.shape[0]), "grid": rm(lab), "interpolation": rm(lab - data.interp),
            "cnn": rm(lab - pred)}
