#!/usr/bin/env python3
"""Throughput of the radar receive path on one MI355X.

Workload: 1024 x 1024 frames (N subcarriers x M OFDM symbols, complex64,
16-QAM, ZC root 7, eight off-grid Rayleigh targets, SNR 0 dB), DFT-CE with
N_cp = 256, periodic Hann window, 4x zero padding to a 4096 x 4096 float32
periodogram that is written out, top-8 peaks.  One step = radar_frame_process
on a batch of distinct frames already resident in HBM.

Prints one JSON line (rank 0).  The dominant kernel's roofline figures come
from HIP events the library records around each of its stage launches during
the timed region; the CPU baseline times the FP64 oracle on a bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "radar frames/s at 1024x1024 (4x pad), plain FP32 vs BF16-MFMA/CNN at equal RMSE"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak from the unit counts: 256 CUs x 2.4 GHz x 128 FMA lanes per
# clock in packed form x 2 flops; the library is built with packed FP32 off,
# which halves what one instruction can do (64 FMA lanes per clock per CU)
FP32_VECTOR_PEAK_TFLOPS = 256 * 2.4e9 * 128 * 2 / 1e12
FP32_UNPACKED_PEAK_TFLOPS = FP32_VECTOR_PEAK_TFLOPS / 2
FP16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense FP16 matrix-core peak (published, without sparsity)
N, M, PAD, NCP, ROOT_ZC, K = 1024, 1024, 4, 256, 7, 8
# Table I: subcarrier spacing and carrier (Eq. 13-15, 19 units); the
# workload's own N, M and prefix N_cp / N set the bin sizes
DF_HZ, FC_HZ, C_MPS = 240e3, 77e9, 3e8
RANGE_BIN_M = C_MPS / (2 * N * DF_HZ)
VELOCITY_BIN_MPS = C_MPS / (2 * FC_HZ * M * (1 + NCP / N) / DF_HZ)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=128, help="frames per step")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU work budget for the oracle baseline (0 disables it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the figures reported beside the headline (refinement, precision forms, FPS-SFT, "
                         "uneven batch)")
    ap.add_argument("--batch-frames", type=int, default=512,
                    help="frames of the uneven Monte-Carlo batch reported beside the headline (0 skips it)")
    ap.add_argument("--rmse-frames", type=int, default=24,
                    help="frames per SNR point of the equal-RMSE comparison of the forms (0 skips it)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device copies of MIB MiB (calibrates HBM byte counters) and exit")
    return ap.parse_args()


def copy_calibration(mib):
    """Three device-to-device copies of a known size: the FETCH_SIZE / WRITE_SIZE
    counters of this copy kernel convert counter units into bytes."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "bytes_per_copy_each_way": n * 4}))


# sources the range kernel is compiled from: a committed counter summary is
# valid while these are unchanged
K3_SOURCES = ("device_common.hpp", "fft.hpp", "k_frame.hpp")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_03883_amd", "csrc")
    for name in K3_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def k3_flops_per_frame(n=N, m=M, pad=PAD, ncp=NCP):
    """Algorithmic flops of the range stage for one frame, in the 5 n log2 n
    convention with pruned inputs, per Doppler row: the forward N-point DFT of
    the N_cp kept taps (log2 N_cp full stages), the window (2 flops per
    subcarrier), the N'-point inverse DFT of N non-zero values (log2 N full
    stages) and |.|^2 (3 flops per output cell)."""
    ilog2 = lambda v: v.bit_length() - 1
    per_row = 5 * n * ilog2(ncp) + 2 * n + 5 * pad * n * ilog2(n) + 3 * pad * n
    return pad * m * per_row


def measured_traffic(frames):
    """HBM bytes of one range-kernel launch over `frames` frames, from the
    committed rocprofv3 counter summary (per-frame bytes of the launch it
    measured), if that was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "k3_range_power_full_frame_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec["hbm_bytes_per_launch"] / rec["frames_per_launch"] * frames


def cpu_baseline(frames, budget_s):
    """The FP64 oracle on the host: receive path of whole frames until the
    budget is used (at least one frame)."""
    import numpy as np
    from oracle import radar_oracle as O

    t0 = time.perf_counter()
    done = 0
    while True:
        f = frames[done % len(frames)]
        P = O.frame_periodogram(f.Y, f.A, n_pad=PAD * N, m_pad=PAD * M, n_cp=NCP, window_kind=O.WINDOW_HANN,
                                zc_root=ROOT_ZC)
        O.find_peaks(P, K)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    del np
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": done / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} whole {N}x{M} frames (FP64 numpy, single thread), {dt:.1f} s",
            "cpu_model": model, "host_cpu_count": os.cpu_count()}


def time_extras(radar, torch, Yd, Ad, cfg, ws, peaks, n_peaks, status, stream, B, steps, warmup):
    """Figures beside the headline: the same step with sub-cell refinement of
    the k peaks, with threshold detection (Eq. 18), with the periodogram not
    materialised (peaks only), with dense ZC precoding
    (on frames precoded that way), the time-domain frame simulation, in the
    BF16x3, FP16x3 and FP16 matrix-core forms (FP16 also without P), the CNN
    refiner, and FPS-SFT (eight
    directions, K = 8) on the same frames."""
    import dataclasses

    out = {}
    cfg_r = dataclasses.replace(cfg, refine=True)
    P = torch.empty((B, cfg.m_pad, cfg.n_pad), dtype=torch.float32, device=Yd.device)
    for _ in range(warmup):
        radar.frame_process(Yd, Ad, cfg_r, K, P=P, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream)
    radar.timing_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        radar.frame_process(Yd, Ad, cfg_r, K, P=P, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = radar.timing_stop()
    out["with_refinement_frames_per_s"] = B * steps / dt
    out["refine_us_per_frame"] = st["refine"][0] / max(st["refine"][1], 1) * 1e3 / B

    # threshold detection (Eq. 18): the same step keeping only peaks above eta
    cfg_t = dataclasses.replace(cfg, threshold=True, pfa=1e-7, noise_power=1.0)
    wst = radar.new_workspace(radar.workspace_bytes(cfg_t, B, K), Yd.device)
    for _ in range(warmup):
        radar.frame_process(Yd, Ad, cfg_t, K, P=P, workspace=wst, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream)
    radar.timing_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        radar.frame_process(Yd, Ad, cfg_t, K, P=P, workspace=wst, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = radar.timing_stop()
    out["with_threshold_frames_per_s"] = B * steps / dt
    out["threshold_stage_us_per_frame"] = {k: st[k][0] / max(st[k][1], 1) * 1e3 / B for k in ("taps", "peaks")}
    out["threshold_mean_detections"] = float(n_peaks.float().mean())
    del P, wst

    # peaks only (P = NULL): the range stage keeps its row maxima and the
    # peak search recomputes the rows it scans; no periodogram is written
    for _ in range(warmup):
        radar.frame_process(Yd, Ad, cfg, K, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream, materialise=False)
    radar.timing_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        radar.frame_process(Yd, Ad, cfg, K, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream, materialise=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = radar.timing_stop()
    out["peaks_only_frames_per_s"] = B * steps / dt
    out["peaks_only_stage_us_per_frame"] = {k: st[k][0] / max(st[k][1], 1) * 1e3 / B for k in ("range", "peaks")}

    # dense ZC precoding (Eq. 24 read literally): frames whose transmitter
    # applied the dense precoding; the taps kernel folds in its FP64 transform
    # and the division
    from synth import frames as S
    from synth import frames_torch as G

    spec_z = dataclasses.replace(S.spec_full(snr_db=0.0), zc_dense=True)
    drawn = [G.make_frame(spec_z, 2, i, device=Yd.device) for i in range(B)]
    Yz = torch.stack([d[0] for d in drawn])
    Az = torch.stack([d[1] for d in drawn])
    del drawn
    cfg_z = dataclasses.replace(cfg, zc_dense=True)
    wsz = radar.new_workspace(radar.workspace_bytes(cfg_z, B, K), Yd.device)
    P = torch.empty((B, cfg.m_pad, cfg.n_pad), dtype=torch.float32, device=Yd.device)
    for _ in range(warmup):
        radar.frame_process(Yz, Az, cfg_z, K, P=P, workspace=wsz, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream)
    radar.timing_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        radar.frame_process(Yz, Az, cfg_z, K, P=P, workspace=wsz, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = radar.timing_stop()
    if int(status.cpu().max()) != 0:
        raise RuntimeError("device status bits set on the dense-precoded frames")
    out["zc_dense_frames_per_s"] = B * steps / dt
    out["zc_dense_stage_us_per_frame"] = {k: st[k][0] / max(st[k][1], 1) * 1e3 / B
                                          for k in ("taps", "doppler", "range", "peaks")}
    del P, wsz, Yz, Az

    # the time-domain frame simulation (Eq. 1-2, 7-10): B frames of eight
    # moving targets from the same symbols
    gen = torch.Generator(device=Yd.device)
    gen.manual_seed(9)
    tg = torch.rand((B, 8, 4), generator=gen, device=Yd.device)
    tg[:, :, 0] = tg[:, :, 0] * 200.0 + 10.0                      # delays well inside the 256-sample prefix
    tg[:, :, 1] = (tg[:, :, 1] - 0.5) * (cfg.n_sym - 2)          # Doppler over the unambiguous range
    tg[:, :, 2:] = tg[:, :, 2:] - 0.5
    nt = torch.full((B,), 8, dtype=torch.int32, device=Yd.device)
    for _ in range(warmup):
        radar.simulate_frames(Ad, tg, nt, n_guard=cfg.n_cp, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        Ysim, _ = radar.simulate_frames(Ad, tg, nt, n_guard=cfg.n_cp, stream=stream)
    torch.cuda.synchronize()
    out["simulate_frames_per_s_8_targets"] = B * steps / (time.perf_counter() - t0)
    del Ysim, tg, nt

    # the matrix-core precision forms of the range stage, same step
    for name, flag in (("bf16x3", radar.FLAG_BF16X3), ("fp16x3", radar.FLAG_FP16X3), ("fp16", radar.FLAG_FP16)):
        cfg_p = dataclasses.replace(cfg, precision=flag)
        P = torch.empty((B, cfg.m_pad, cfg.n_pad), dtype=torch.float32, device=Yd.device)
        for _ in range(warmup):
            radar.frame_process(Yd, Ad, cfg_p, K, P=P, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                                stream=stream)
        radar.timing_start(steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            radar.frame_process(Yd, Ad, cfg_p, K, P=P, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                                stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = radar.timing_stop()
        out[f"{name}_frames_per_s"] = B * steps / dt
        out[f"{name}_stage_us_per_frame"] = {k: st[k][0] / max(st[k][1], 1) * 1e3 / B
                                             for k in ("taps", "doppler", "range", "peaks")}
        del P

    # the FP16 form without P: its matrix-core row maxima choose the rows and
    # the peak search rescans them in FP32 (the FP32 periodogram's peaks)
    cfg_p = dataclasses.replace(cfg, precision=radar.FLAG_FP16)
    for _ in range(warmup):
        radar.frame_process(Yd, Ad, cfg_p, K, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream, materialise=False)
    radar.timing_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        radar.frame_process(Yd, Ad, cfg_p, K, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream, materialise=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = radar.timing_stop()
    out["fp16_peaks_only_frames_per_s"] = B * steps / dt
    out["fp16_peaks_only_stage_us_per_frame"] = {k: st[k][0] / max(st[k][1], 1) * 1e3 / B
                                                 for k in ("taps", "doppler", "range", "peaks")}

    # the CNN refiner: inference on 8192 patches cut from the benchmark frames'
    # periodograms around their peaks (the frames' 32 x 8 patches, tiled), and
    # one training step of 256 patches
    import numpy as np
    from synth import cnn_init

    P = torch.empty((B, cfg.m_pad, cfg.n_pad), dtype=torch.float32, device=Yd.device)
    radar.frame_process(Yd, Ad, cfg, K, P=P, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                        stream=stream)
    pat, _ = radar.cnn_patches(P, peaks, n_peaks)
    del P
    nb = 8192
    pat = pat.repeat((nb + pat.shape[0] - 1) // pat.shape[0], 1, 1)[:nb].contiguous()
    theta = torch.from_numpy(cnn_init.init_params(0)).to(Yd.device)
    cws = radar.CnnWorkspace(nb, False, Yd.device)
    for _ in range(warmup):
        radar.cnn_forward(theta, pat, workspace=cws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        radar.cnn_forward(theta, pat, workspace=cws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    flops = 11247656  # per patch: conv1 589824, conv2 4718592, conv3 4718592, conv4 1179648, dense 41000
    out["cnn_inference"] = {"patches": nb, "ms": dt * 1e3, "patches_per_s": nb / dt,
                            "tflops": nb * flops / dt / 1e12, "mfma_bf16_peak_tflops": 2500.0}
    tws = radar.CnnWorkspace(256, True, Yd.device)
    lab = torch.zeros((256, 2), dtype=torch.float32, device=Yd.device)
    mom, vel = torch.zeros_like(theta), torch.zeros_like(theta)
    loss = torch.empty(1, dtype=torch.float32, device=Yd.device)
    xb = pat[:256].contiguous()
    for t in range(warmup):
        radar.cnn_train_step(theta, mom, vel, t + 1, 1e-3, xb, lab, loss, workspace=tws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(steps):
        radar.cnn_train_step(theta, mom, vel, warmup + t + 1, 1e-3, xb, lab, loss, workspace=tws)
    torch.cuda.synchronize()
    out["cnn_train_step_ms_batch256"] = (time.perf_counter() - t0) / steps * 1e3
    # the whole FP32 path followed by the CNN on every frame's k peaks (patches cut from P, inference)
    P = torch.empty((B, cfg.m_pad, cfg.n_pad), dtype=torch.float32, device=Yd.device)
    cws_f = radar.CnnWorkspace(B * K, False, Yd.device)

    def cnn_step():
        radar.frame_process(Yd, Ad, cfg, K, P=P, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream)
        pt, _ = radar.cnn_patches(P, peaks, n_peaks, stream=stream)
        radar.cnn_forward(theta, pt, workspace=cws_f, stream=stream)

    for _ in range(warmup):
        cnn_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cnn_step()
    torch.cuda.synchronize()
    out["with_cnn_frames_per_s"] = B * steps / (time.perf_counter() - t0)
    del P, np

    sft = radar.sft_desc(K)
    ws_sft = radar.new_workspace(radar.sft_workspace_bytes(cfg, sft, B), Yd.device)
    for _ in range(warmup):
        radar.fps_sft(Yd, Ad, cfg, sft, workspace=ws_sft, stream=stream)
    radar.timing_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        radar.fps_sft(Yd, Ad, cfg, sft, workspace=ws_sft, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = radar.timing_stop()
    out["fps_sft_frames_per_s"] = B * steps / dt
    out["fps_sft_us_per_frame"] = {k: st[k][0] / max(st[k][1], 1) * 1e3 / B for k in ("sft_slices", "sft_decode")}
    del ws_sft
    # FPS-SFT on Table I's frame, N = 2048 by M = 560 (Q = lcm = 71680, the
    # prime-factor path): 32 frames of eight off-grid targets at 10 dB
    from synth import frames as S
    from synth import frames_torch as G

    spec = S.FrameSpec(n_sub=2048, n_sym=560, qam=16, zc_root=7, n_targets=8, snr_db=10.0, on_grid=False,
                       rho_min=1.0, rho_max=511.0, nu_abs_max=279.0, rayleigh=True, min_sep=3.0)
    drawn = [G.make_frame(spec, 99, i, device=Yd.device) for i in range(32)]
    Yt = torch.stack([d[0] for d in drawn])
    At = torch.stack([d[1] for d in drawn])
    del drawn
    cfg_t1 = radar.Config(2048, 560, 2048, 560, 2048, zc_root=7)
    ws_t1 = radar.new_workspace(radar.sft_workspace_bytes(cfg_t1, sft, 32), Yd.device)
    for _ in range(warmup):
        radar.fps_sft(Yt, At, cfg_t1, sft, workspace=ws_t1, stream=stream)
    radar.timing_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        radar.fps_sft(Yt, At, cfg_t1, sft, workspace=ws_t1, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = radar.timing_stop()
    out["fps_sft_table1_2048x560_frames_per_s"] = 32 * steps / dt
    out["fps_sft_table1_us_per_frame"] = {k: st[k][0] / max(st[k][1], 1) * 1e3 / 32
                                          for k in ("sft_slices", "sft_decode")}
    del Yt, At, ws_t1
    print(f"[bench] extras {out}", file=sys.stderr, flush=True)
    return out


def _match_errors(truth_rho, truth_nu, det, n, m):
    """Range and Doppler errors (native bins) of the truth-to-detection
    assignment minimising the summed wrapped distance."""
    import numpy as np
    from scipy.optimize import linear_sum_assignment

    if not det:
        return []
    dr = np.array([[r - tr for r, _ in det] for tr in truth_rho])
    dv = np.array([[v - tv for _, v in det] for tv in truth_nu])
    dv = (dv + m / 2) % m - m / 2
    rows, cols = linear_sum_assignment(np.hypot(dr, dv))
    return [(dr[i, j], dv[i, j]) for i, j in zip(rows, cols)]


def rmse_comparison(radar, torch, dev, fps, per_snr=24, train_frames=768, train_steps=1500):
    """Range and velocity RMSE of every form on the same frames: the full-frame
    workload's generator at SNR -20, -15, ..., 10 dB (per_snr frames each,
    eight off-grid Rayleigh targets), top-8 peaks, each truth matched to a
    detection by the assignment of least wrapped distance; a hit has both
    errors within one native bin, RMSE over hits (Eq. 19 units and native
    bins), hit rate beside it.  The forms: the FP32 grid peak, FP32 with the
    interpolation refinement, the grid peaks of the three matrix-core range
    forms, the FP16 form without P (its rows rescanned in FP32), and FP32
    with the CNN refiner (trained here, by the library's own
    kernels, on train_frames frames of the same workload drawn from other
    seeds).  fps: each form's frames/s on the benchmark batch."""
    import dataclasses

    import numpy as np

    from paper_2209_03883_amd import cnn_train
    from synth import cnn_init
    from synth import frames as S
    from synth import frames_torch as G

    data = cnn_train.make_patches(train_frames, 12, n=N, m=M, k=K, chunk=32, device=dev)
    theta, _ = cnn_train.train(cnn_init.init_params(0), data, train_steps, device=dev)
    del data
    base = radar.Config(N, M, PAD * N, PAD * M, NCP, zc_root=ROOT_ZC, window=radar.WIN_HANN)
    forms = {
        "fp32_grid": dict(),
        "fp32_refined": dict(refine=True),
        "bf16x3_grid": dict(precision=radar.FLAG_BF16X3),
        "fp16x3_grid": dict(precision=radar.FLAG_FP16X3),
        "fp16_grid": dict(precision=radar.FLAG_FP16),
        "fp16_peaks_only_grid": dict(precision=radar.FLAG_FP16),  # P not written, rows rescanned in FP32
        "fp32_cnn": dict(),
    }
    snrs = [-20.0, -15.0, -10.0, -5.0, 0.0, 5.0, 10.0]
    acc = {f: {s: [[], [], 0] for s in snrs} for f in forms}
    same_cells = {f: [0, 0] for f in forms}
    for si, snr in enumerate(snrs):
        drawn = [G.make_frame(S.spec_full(snr_db=snr), 21, si * 1000 + i, device=dev) for i in range(per_snr)]
        Y = torch.stack([d[0] for d in drawn])
        A = torch.stack([d[1] for d in drawn])
        truth = [d[2] for d in drawn]
        del drawn
        grid32 = {}
        for name, kw in forms.items():
            P, peaks, n_peaks, st = radar.frame_process(Y, A, dataclasses.replace(base, **kw), K,
                                                        materialise=name != "fp16_peaks_only_grid")
            off = None
            if name == "fp32_cnn":
                pt, _ = radar.cnn_patches(P, peaks, n_peaks)
                off = cnn_train.predict(theta, pt).cpu().numpy().reshape(per_snr, K, 2)
            pk = radar.unpack_peaks(peaks, n_peaks.cpu())
            del P
            for f in range(per_snr):
                cells = [(s, r) for s, r, *_ in pk[f]]
                if name == "fp32_grid":
                    grid32[f] = cells
                else:
                    same_cells[name][0] += int(cells == grid32[f])
                    same_cells[name][1] += 1
                det = []
                for i, (s, r, _, so, ro) in enumerate(pk[f]):
                    if name == "fp32_refined":
                        det.append(((r + ro) / PAD, (s + so) / PAD))
                    elif name == "fp32_cnn":
                        det.append(((r + off[f, i, 0]) / PAD, (s + off[f, i, 1]) / PAD))
                    else:
                        det.append((r / PAD, s / PAD))
                e = acc[name][snr]
                for er, ev in _match_errors(truth[f][0], truth[f][1], det, N, M):
                    if abs(er) <= 1.0 and abs(ev) <= 1.0:
                        e[0].append(er)
                        e[1].append(ev)
                e[2] += len(truth[f][0])
        del Y, A

    def rm(v):
        return float(np.sqrt(np.mean(np.square(v)))) if v else None

    out = {"snr_db": snrs, "frames_per_snr": per_snr, "range_bin_m": RANGE_BIN_M,
           "velocity_bin_mps": VELOCITY_BIN_MPS, "cnn_training": {"frames": train_frames, "steps": train_steps},
           "forms": {}}
    for name in forms:
        er = [x for s in snrs for x in acc[name][s][0]]
        ev = [x for s in snrs for x in acc[name][s][1]]
        tot = sum(acc[name][s][2] for s in snrs)
        out["forms"][name] = {
            "frames_per_s": fps.get(name),
            "rmse_range_m": rm(er) * RANGE_BIN_M if er else None,
            "rmse_velocity_mps": rm(ev) * VELOCITY_BIN_MPS if ev else None,
            "rmse_range_bins": rm(er), "rmse_doppler_bins": rm(ev), "hit_rate": len(er) / max(tot, 1),
            "per_snr": {f"{s:+.0f} dB": {"hit_rate": len(acc[name][s][0]) / max(acc[name][s][2], 1),
                                         "rmse_range_bins": rm(acc[name][s][0]),
                                         "rmse_doppler_bins": rm(acc[name][s][1])} for s in snrs},
        }
        if name != "fp32_grid":
            out["forms"][name]["frames_with_fp32_grid_cells"] = same_cells[name][0] / max(same_cells[name][1], 1)
    g = out["forms"]["fp32_grid"]
    for name, v in out["forms"].items():
        if v["rmse_range_bins"] and g["rmse_range_bins"]:
            v["rmse_ratio_to_fp32_grid"] = [v["rmse_range_bins"] / g["rmse_range_bins"],
                                            v["rmse_doppler_bins"] / g["rmse_doppler_bins"]]
    return out


def device_copy_gbs(torch, dev, mib=2048, reps=5):
    """Bandwidth of a plain device-to-device copy of `mib` MiB (read + write
    bytes over time, HIP events): the practical HBM ceiling beside the 8 TB/s
    datasheet figure."""
    n = mib * (1 << 20) // 4
    src = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 4 * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
    del src, dst
    return gbs


def time_batch(radar, torch, n_frames, steps):
    """The uneven Monte-Carlo batch: n_frames frames of random N x M shapes in
    one autotuned, graph-captured plan (4x padding both axes, N_cp = N/4, Hann,
    k = 16); throughput over replays, and range / Doppler RMSE against SNR
    from the grid peaks and from the refined peaks."""
    import numpy as np
    from synth import frames_torch as G

    specs = G.monte_carlo_specs(n_frames)
    jobs, truth = [], []
    for i, sp in enumerate(specs):
        Y, A, tgt = G.make_frame(sp, 3, i)
        cfg = radar.Config(sp.n_sub, sp.n_sym, 4 * sp.n_sub, 4 * sp.n_sym, sp.n_sub // 4, zc_root=7,
                           window=radar.WIN_HANN)
        jobs.append((Y, A, cfg, 16))
        truth.append(tgt)
    torch.cuda.synchronize()
    b = radar.Batch(jobs, graph=True, tune=True)
    b.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.launch()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    alg = sum(80 * sp.n_sub * sp.n_sym for sp in specs)

    def rmse_table(batch):
        bins = {}
        for i, sp in enumerate(specs):
            _, pk, st = batch.results(i)
            n, m = sp.n_sub, sp.n_sym
            det = [((r + ro) * n / (4 * n), (s + so) * m / (4 * m)) for s, r, _, so, ro in pk[:sp.n_targets]]
            errs = _match_errors(truth[i][0], truth[i][1], det, n, m)
            key = int(np.floor((sp.snr_db + 20.0) / 5.0)) * 5 - 20
            e = bins.setdefault(key, [[], [], 0])
            for er, ev in errs:
                if abs(er) <= 1.0 and abs(ev) <= 1.0:  # a hit: both errors within one native bin
                    e[0].append(er)
                    e[1].append(ev)
            e[2] += sp.n_targets
        out = {}
        for key in sorted(bins):
            er, ev, tot = bins[key]
            out[f"{key}..{key + 5} dB"] = {
                "targets": tot, "hit_rate": len(er) / max(tot, 1),
                "rmse_range_bins_hits": float(np.sqrt(np.mean(np.square(er)))) if er else None,
                "rmse_doppler_bins_hits": float(np.sqrt(np.mean(np.square(ev)))) if ev else None}
        return out

    grid = rmse_table(b)
    groups = b.groups()
    plans = b.plans()
    b.close()
    del b
    rjobs = [(Y, A, dataclasses_replace(cfg, refine=True), k) for Y, A, cfg, k in jobs]
    br = radar.Batch(rjobs, graph=True, tune=True)
    br.launch()
    torch.cuda.synchronize()
    refined = rmse_table(br)
    br.close()
    return {"batch_frames": n_frames, "batch_shape_groups": len(groups),
            "batch_frames_per_s": n_frames / dt, "batch_ms_per_launch": dt * 1e3,
            "batch_algorithmic_gbytes": alg / 1e9, "batch_hbm_gbs": alg / dt / 1e9,
            "batch_tuned_plans": {"groups": len(plans),
                                  "two_per_cu": sum(1 for p in plans if p["k3_mult"] == 2 or p["k1_mult"] == 2),
                                  "per_row_range_kernel": sum(p["k3_generic"] for p in plans),
                                  "half_doppler_tiles": sum(p["k2_half_tile"] for p in plans),
                                  "scan_128_per_frame": sum(1 for p in plans if p["scan_groups"] == 128)},
            "batch_rmse_vs_snr_grid": grid, "batch_rmse_vs_snr_refined": refined}


def fp16_range_hbm(extras, copy_gbs):
    """The FP16 matrix-core form's range stage against HBM: its algorithmic
    bytes per frame (read U, write P) over its HIP-event time per frame."""
    st = extras.get("fp16_stage_us_per_frame")
    if not st or not st.get("range"):
        return {}
    gbs = (PAD * M * NCP * 8 + PAD * M * PAD * N * 4) / (st["range"] * 1e-6) / 1e9
    return {"fp16_range_hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                               "frac_of_device_copy": gbs / copy_gbs}}


def fp16_peaks_only_range_mfma(extras):
    """The FP16 form's store-free range kernel (peaks only) against the FP16
    matrix-core peak: its issued matrix-core work per frame, 58
    v_mfma_f32_32x32x16_f16 per Doppler row (f1 2, f2 8, and i1 8 + i2 8 for
    each of three phases) of 2 x 32 x 32 x 16 flops each, over its HIP-event
    time per frame.  These are the flops the matrix cores execute (dense 32-point
    DFTs by matrix product), not the FFT's 5 n log2 n count."""
    st = extras.get("fp16_peaks_only_stage_us_per_frame")
    if not st or not st.get("range"):
        return {}
    flops = 58 * 2 * 32 * 32 * 16 * PAD * M
    tf = flops / (st["range"] * 1e-6) / 1e12
    return {"fp16_peaks_only_range_mfma": {"achieved": tf, "peak": FP16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                           "frac": tf / FP16_MFMA_PEAK_TFLOPS}}


def dataclasses_replace(cfg, **kw):
    import dataclasses

    return dataclasses.replace(cfg, **kw)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the radar path runs one "
              "frame per GPU without collectives, so multi-GPU throughput is N x this figure by design "
              "and is not measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2209_03883_amd import radar
    from synth import frames as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    B = args.frames
    print(f"[bench] generating {B} frames", file=sys.stderr, flush=True)
    # the frames are drawn on the GPU (same recipe and seeds as the host generator)
    from synth import frames_torch as G

    drawn = [G.make_frame(S.spec_full(snr_db=0.0), 2, i, device=dev) for i in range(B)]
    Yd = torch.stack([d[0] for d in drawn])
    Ad = torch.stack([d[1] for d in drawn])
    del drawn
    cfg = radar.Config(N, M, PAD * N, PAD * M, NCP, zc_root=ROOT_ZC, window=radar.WIN_HANN)
    P = torch.empty((B, PAD * M, PAD * N), dtype=torch.float32, device=dev)
    ws = radar.new_workspace(radar.workspace_bytes(cfg, B, K), dev)
    peaks = radar.alloc_peaks(B, K, dev)
    n_peaks = torch.zeros(B, dtype=torch.int32, device=dev)
    status = torch.zeros(B, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        radar.frame_process(Yd, Ad, cfg, K, P=P, workspace=ws, peaks=peaks, n_peaks=n_peaks, status=status,
                            stream=stream)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if int(status.cpu().max()) != 0:
        raise RuntimeError("device status bits set on the benchmark frames")

    radar.timing_start(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = radar.timing_stop()
    print(f"[bench] timed {args.steps} steps in {dt:.3f} s; stages {stages}", file=sys.stderr, flush=True)

    extras = {} if args.no_extras else time_extras(radar, torch, Yd, Ad, cfg, ws, peaks, n_peaks, status, stream,
                                                   B, args.steps, args.warmup)
    if not args.no_extras and args.batch_frames > 0:
        print(f"[bench] uneven batch of {args.batch_frames} frames", file=sys.stderr, flush=True)
        extras.update(time_batch(radar, torch, args.batch_frames, 5))
        print(f"[bench] batch {({k: v for k, v in extras.items() if k.startswith('batch_') and 'rmse' not in k})}",
              file=sys.stderr, flush=True)

    frames_done = B * args.steps
    fps = frames_done / dt
    if not args.no_extras and args.rmse_frames > 0:
        print("[bench] equal-RMSE comparison of the forms", file=sys.stderr, flush=True)
        fps_forms = {"fp32_grid": fps, "fp32_refined": extras.get("with_refinement_frames_per_s"),
                     "bf16x3_grid": extras.get("bf16x3_frames_per_s"),
                     "fp16x3_grid": extras.get("fp16x3_frames_per_s"),
                     "fp16_grid": extras.get("fp16_frames_per_s"),
                     "fp16_peaks_only_grid": extras.get("fp16_peaks_only_frames_per_s"),
                     "fp32_cnn": extras.get("with_cnn_frames_per_s")}
        extras["equal_rmse"] = rmse_comparison(radar, torch, dev, fps_forms, per_snr=args.rmse_frames)
    copy_gbs = device_copy_gbs(torch, dev)
    rng_ms, rng_n = stages["range"]
    k3_ms = rng_ms / max(rng_n, 1)
    # algorithmic bytes of one range-kernel launch: read the Doppler-tap rows
    # U [M'][N_cp] complex64 and write P [M'][N'] float32, per frame
    k3_bytes = B * (PAD * M * NCP * 8 + PAD * M * PAD * N * 4)
    achieved = k3_bytes / (k3_ms * 1e-3) / 1e9
    # the range kernel is bound by its FP32 vector instructions, not by HBM
    k3_tflops = B * k3_flops_per_frame() / (k3_ms * 1e-3) / 1e12
    traffic = measured_traffic(B)

    out = {
        "metric": METRIC,
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"frame {N}x{M} complex64 -> DFT-CE (N_cp={NCP}) -> {PAD * N}x{PAD * M} float32 "
                        f"periodogram (4x zero padding, Hann) -> top-{K} peaks; 16-QAM, ZC root {ROOT_ZC}, "
                        "8 off-grid Rayleigh targets, SNR 0 dB",
            "frames_per_step": B,
            "periodogram_materialised": True,
            "hbm_roofline_frames_per_s": HBM_PEAK_GBS * 1e9 / (16 * N * M + 4 * PAD * N * PAD * M),
            "hbm_frac": fps / (HBM_PEAK_GBS * 1e9 / (16 * N * M + 4 * PAD * N * PAD * M)),
            "device_copy_gbs": copy_gbs,
            "k3_frac_of_device_copy": achieved / copy_gbs,
            "k3_hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS},
            "k3_frac_of_unpacked_fp32": k3_tflops / FP32_UNPACKED_PEAK_TFLOPS,
            **fp16_range_hbm(extras, copy_gbs),
            **fp16_peaks_only_range_mfma(extras),
            "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1]},
            **extras,
        },
        "roofline": {
            "kernel": "k3_range_power",
            "bound": "alu",
            "achieved": k3_tflops,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": k3_tflops / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
        },
    }
    if args.cpu_seconds > 0:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline([S.make_frame(S.spec_full(snr_db=0.0), 2, i) for i in range(2)],
                                           args.cpu_seconds)
    print(json.dumps(out), flush=True)
    del np


if __name__ == "__main__":
    main()
