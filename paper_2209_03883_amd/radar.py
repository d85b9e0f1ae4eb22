"""Python binding of libradar (include/radar.h).

Argument marshalling only: every step of the receive path runs in the HIP
library.  torch supplies device memory and the stream; it computes nothing
here.  The binding refuses to run when the library is not built.
"""

from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RADAR_LIB_PATH") or os.path.join(PKG_DIR, "libradar.so")

RADAR_OK = 0
RADAR_E_ARG = -1
RADAR_E_UNSUPPORTED = -2
RADAR_E_WORKSPACE = -3
RADAR_E_HIP = -4
RADAR_E_NOT_COPRIME = -5

WIN_RECT, WIN_HANN, WIN_HAMMING = 0, 1, 2
ZC_NONE, ZC_DIAG, ZC_DENSE = 0, 1, 2
ST_ZERO_SYMBOL, ST_NONFINITE, ST_ISI = 1, 2, 4
FLAG_REFINE, FLAG_BF16X3, FLAG_FP16X3, FLAG_THRESHOLD, FLAG_FP16 = 1, 2, 4, 8, 16

EXPORTED = (
    "radar_version", "radar_status_string", "radar_init",
    "radar_frame_workspace_size", "radar_frame_process", "radar_periodogram",
    "radar_detect_workspace_size", "radar_detect_topk", "radar_timing_start", "radar_timing_stop",
    "radar_sft_default", "radar_fps_sft_workspace_size", "radar_fps_sft",
    "radar_batch_workspace_size", "radar_batch_create", "radar_batch_launch", "radar_batch_info", "radar_batch_plan",
    "radar_batch_destroy",
    "radar_cnn_param_count", "radar_cnn_workspace_size", "radar_cnn_patches", "radar_cnn_forward",
    "radar_cnn_gradient", "radar_cnn_adam", "radar_cnn_train_step", "radar_tap_wiener_weights",
    "radar_simulate_frames", "radar_papr", "radar_hpa", "radar_frame_process_noalloc",
)
BATCH_GRAPH, BATCH_TUNE = 1, 2
STAGES = ("taps", "doppler", "range", "peaks", "refine", "sft_slices", "sft_decode")


class RadarError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} ({code})")


class FrameDesc(ctypes.Structure):
    _fields_ = [
        ("n_sub", ctypes.c_int32), ("n_sym", ctypes.c_int32),
        ("n_pad", ctypes.c_int32), ("m_pad", ctypes.c_int32),
        ("n_cp", ctypes.c_int32), ("zc_mode", ctypes.c_int32),
        ("zc_root", ctypes.c_int32), ("zc_shift", ctypes.c_int32),
        ("window", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("ld", ctypes.c_int64),
        ("pfa", ctypes.c_float), ("noise_power", ctypes.c_float),
        ("tap_weights", ctypes.c_void_p),
    ]


class Peak(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("r", ctypes.c_int32), ("p", ctypes.c_float),
                ("s_off", ctypes.c_float), ("r_off", ctypes.c_float)]


PEAK_WORDS = ctypes.sizeof(Peak) // 4  # 5 x 32-bit words


class SimDesc(ctypes.Structure):
    _fields_ = [
        ("n_sub", ctypes.c_int32), ("n_sym", ctypes.c_int32), ("n_guard", ctypes.c_int32),
        ("max_targets", ctypes.c_int32), ("ld", ctypes.c_int64), ("fc_over_df", ctypes.c_double),
    ]


class FrameJob(ctypes.Structure):
    _fields_ = [("d", FrameDesc), ("Y", ctypes.c_void_p), ("A", ctypes.c_void_p), ("P", ctypes.c_void_p),
                ("peaks", ctypes.c_void_p), ("n_peaks", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("k", ctypes.c_int32)]


class SftDesc(ctypes.Structure):
    _fields_ = [("n_dirs", ctypes.c_int32), ("dirs", (ctypes.c_int32 * 2) * 16), ("k", ctypes.c_int32),
                ("pfa", ctypes.c_float), ("tol", ctypes.c_float), ("flags", ctypes.c_int32)]

_lib = None


def lib() -> ctypes.CDLL:
    """Load libradar.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2209_03883_amd.build_lib")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    dp = ctypes.POINTER(FrameDesc)
    L.radar_version.restype = ctypes.c_int
    L.radar_status_string.restype = ctypes.c_char_p
    L.radar_status_string.argtypes = [ctypes.c_int]
    L.radar_init.restype = ctypes.c_int
    L.radar_frame_workspace_size.restype = sz
    L.radar_frame_workspace_size.argtypes = [dp, i32, i32]
    L.radar_frame_process.restype = ctypes.c_int
    L.radar_frame_process.argtypes = [dp, i32, vp, vp, i64, vp, i64, i32, vp, vp, vp, vp, sz, vp]
    L.radar_frame_process_noalloc.restype = ctypes.c_int
    L.radar_frame_process_noalloc.argtypes = [dp, i32, vp, vp, i64, vp, i64, i32, vp, vp, vp, vp]
    L.radar_periodogram.restype = ctypes.c_int
    L.radar_periodogram.argtypes = [dp, i32, vp, i64, vp, i64, vp, sz, vp]
    L.radar_detect_workspace_size.restype = sz
    L.radar_detect_workspace_size.argtypes = [i32, i32, i32, i32]
    L.radar_detect_topk.restype = ctypes.c_int
    L.radar_detect_topk.argtypes = [vp, i32, i32, i32, i64, i32, vp, vp, vp, sz, vp]
    sp = ctypes.POINTER(SftDesc)
    L.radar_sft_default.restype = None
    L.radar_sft_default.argtypes = [sp, i32]
    L.radar_fps_sft_workspace_size.restype = sz
    L.radar_fps_sft_workspace_size.argtypes = [dp, sp, i32]
    L.radar_fps_sft.restype = ctypes.c_int
    L.radar_fps_sft.argtypes = [dp, sp, i32, vp, vp, i64, vp, vp, vp, vp, vp, sz, vp]
    jp = ctypes.POINTER(FrameJob)
    L.radar_batch_workspace_size.restype = sz
    L.radar_batch_workspace_size.argtypes = [jp, i32]
    L.radar_batch_create.restype = ctypes.c_int
    L.radar_batch_create.argtypes = [jp, i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
    L.radar_batch_launch.restype = ctypes.c_int
    L.radar_batch_launch.argtypes = [vp, vp]
    L.radar_batch_info.restype = ctypes.c_int
    ip = ctypes.POINTER(i32)
    L.radar_batch_info.argtypes = [vp, i32, ip, ip, ip, ip, ip]
    L.radar_batch_plan.restype = ctypes.c_int
    L.radar_batch_plan.argtypes = [vp, i32, ip, ip]
    L.radar_batch_destroy.restype = None
    L.radar_batch_destroy.argtypes = [vp]
    fp = ctypes.c_void_p
    L.radar_hpa.restype = ctypes.c_int
    L.radar_hpa.argtypes = [i32, i32, i64, i32, vp, i64, ctypes.c_double, vp, vp]
    L.radar_papr.restype = ctypes.c_int
    L.radar_papr.argtypes = [i32, i32, i64, i32, vp, i64, vp, vp]
    L.radar_simulate_frames.restype = ctypes.c_int
    L.radar_simulate_frames.argtypes = [ctypes.POINTER(SimDesc), i32, vp, i64, vp, vp, vp, vp, vp, vp]
    L.radar_tap_wiener_weights.restype = ctypes.c_int
    L.radar_tap_wiener_weights.argtypes = [ctypes.POINTER(ctypes.c_double), i32, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_float)]
    L.radar_cnn_param_count.restype = i32
    L.radar_cnn_workspace_size.restype = sz
    L.radar_cnn_workspace_size.argtypes = [i32, i32]
    L.radar_cnn_patches.restype = ctypes.c_int
    L.radar_cnn_patches.argtypes = [fp, i64, i32, i32, i32, i32, vp, vp, fp, vp, vp]
    L.radar_cnn_forward.restype = ctypes.c_int
    L.radar_cnn_forward.argtypes = [fp, fp, i32, fp, vp, sz, vp]
    L.radar_cnn_gradient.restype = ctypes.c_int
    L.radar_cnn_gradient.argtypes = [fp, fp, fp, i32, fp, fp, vp, sz, vp]
    L.radar_cnn_adam.restype = ctypes.c_int
    L.radar_cnn_adam.argtypes = [fp, fp, fp, fp, i32, ctypes.c_float, vp]
    L.radar_cnn_train_step.restype = ctypes.c_int
    L.radar_cnn_train_step.argtypes = [fp, fp, fp, i32, ctypes.c_float, fp, fp, i32, fp, vp, sz, vp]
    L.radar_timing_start.restype = ctypes.c_int
    L.radar_timing_start.argtypes = [i32]
    L.radar_timing_stop.restype = ctypes.c_int
    L.radar_timing_stop.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    _lib = L
    return L


def status_string(code: int) -> str:
    return lib().radar_status_string(int(code)).decode()


def _check(code: int, where: str):
    if code != RADAR_OK:
        raise RadarError(code, where)


@dataclass
class Config:
    """One frame shape (the fields of radar_frame_desc)."""

    n_sub: int
    n_sym: int
    n_pad: int
    m_pad: int
    n_cp: int
    zc_root: int | None = None
    zc_shift: int = 0
    window: int = WIN_HANN
    refine: bool = False
    precision: int = 0          # 0 (FP32), FLAG_BF16X3, FLAG_FP16X3 or FLAG_FP16
    threshold: bool = False     # Eq. 18 detection (pfa, noise_power)
    pfa: float = 1e-2
    noise_power: float = 0.0
    zc_dense: bool = False      # Eq. 24 read literally (L = N^2) instead of the diagonal reading
    tap_weights: torch.Tensor | None = None  # n_cp float32 on the device: LMMSE-based DFT-CE

    def desc(self, ld: int | None = None) -> FrameDesc:
        return FrameDesc(self.n_sub, self.n_sym, self.n_pad, self.m_pad, self.n_cp,
                         ZC_NONE if self.zc_root is None else (ZC_DENSE if self.zc_dense else ZC_DIAG),
                         0 if self.zc_root is None else int(self.zc_root), int(self.zc_shift),
                         int(self.window),
                         (FLAG_REFINE if self.refine else 0) | int(self.precision)
                         | (FLAG_THRESHOLD if self.threshold else 0),
                         int(self.n_sub if ld is None else ld), float(self.pfa), float(self.noise_power),
                         self._tap_weights_ptr())

    def _tap_weights_ptr(self):
        w = self.tap_weights
        if w is None:
            return None
        if w.dtype != torch.float32 or w.dim() != 1 or w.numel() != self.n_cp or not w.is_contiguous():
            raise ValueError("tap_weights must be a contiguous float32 vector of n_cp entries")
        return w.data_ptr()


def _stream_ptr(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _as_frames(x: torch.Tensor, cfg: Config, name: str) -> torch.Tensor:
    if not x.is_cuda or x.dtype != torch.complex64:
        raise TypeError(f"{name} must be a complex64 CUDA tensor")
    if x.dim() == 2:
        x = x.unsqueeze(0)
    if x.dim() != 3 or tuple(x.shape[1:]) != (cfg.n_sym, cfg.n_sub):
        raise ValueError(f"{name} must have shape (F, {cfg.n_sym}, {cfg.n_sub})")
    if x.stride(2) != 1 or x.stride(1) < cfg.n_sub:
        raise ValueError(f"{name} must have contiguous subcarriers")
    return x


def _frame_stride(x: torch.Tensor) -> int:
    return int(x.stride(0)) if x.shape[0] > 1 else int(x.shape[1] * x.stride(1))


def simulate_frames(A: torch.Tensor, targets: torch.Tensor, n_targets: torch.Tensor, *, n_guard: int,
                    fc_over_df: float = 77e9 / 240e3, noise: torch.Tensor | None = None, stream=None):
    """radar_simulate_frames: received frames (F, M, N) complex64 from the
    time-domain model, and the per-frame status words.

    A: (F, M, N) complex64 CUDA (contiguous rows); targets: (F, T, 4) float32
    CUDA rows (rho, nu, b_re, b_im); n_targets: (F,) int32 CUDA."""
    L = lib()
    if A.dim() == 2:
        A = A[None]
    if not A.is_cuda or A.dtype != torch.complex64 or A.stride(2) != 1:
        raise TypeError("A must be a complex64 CUDA tensor (F, M, N) with contiguous rows")
    if targets.dtype != torch.float32 or targets.dim() != 3 or targets.shape[2] != 4 or not targets.is_contiguous():
        raise TypeError("targets must be a contiguous float32 tensor (F, T, 4)")
    if n_targets.dtype != torch.int32 or n_targets.numel() != A.shape[0]:
        raise TypeError("n_targets must be int32 with one entry per frame")
    F, M, N = A.shape
    Y = torch.empty((F, M, N), dtype=torch.complex64, device=A.device)
    status = torch.zeros(F, dtype=torch.int32, device=A.device)
    if noise is not None and (noise.shape != Y.shape or noise.dtype != torch.complex64 or not noise.is_contiguous()):
        raise TypeError("noise must be a contiguous complex64 tensor shaped like A")
    if A.stride() != Y.stride():
        A = A.contiguous()
    d = SimDesc(N, M, int(n_guard), int(targets.shape[1]), int(A.stride(1)), float(fc_over_df))
    _check(L.radar_simulate_frames(ctypes.byref(d), F, A.data_ptr(), int(A.stride(0)), targets.data_ptr(),
                                   n_targets.data_ptr(), None if noise is None else noise.data_ptr(), Y.data_ptr(),
                                   status.data_ptr(), _stream_ptr(stream)), "radar_simulate_frames")
    return Y, status


def hpa(A: torch.Tensor, q_db: float = 2.0, stream=None) -> torch.Tensor:
    """radar_hpa: the Eq. 26 amplifier on (F, M, N) complex64 CUDA symbols; a new tensor."""
    L = lib()
    if A.dim() == 2:
        A = A[None]
    if not A.is_cuda or A.dtype != torch.complex64 or not A.is_contiguous():
        raise TypeError("A must be a contiguous complex64 CUDA tensor (F, M, N)")
    F, M, N = A.shape
    out = torch.empty_like(A)
    _check(L.radar_hpa(N, M, int(A.stride(1)), F, A.data_ptr(), int(A.stride(0)), float(q_db), out.data_ptr(),
                       _stream_ptr(stream)), "radar_hpa")
    return out


def papr(A: torch.Tensor, stream=None) -> torch.Tensor:
    """radar_papr: Eq. 25 per symbol of (F, M, N) complex64 CUDA symbols, (F, M) float32 linear."""
    L = lib()
    if A.dim() == 2:
        A = A[None]
    if not A.is_cuda or A.dtype != torch.complex64 or A.stride(2) != 1:
        raise TypeError("A must be a complex64 CUDA tensor (F, M, N) with contiguous rows")
    F, M, N = A.shape
    out = torch.empty((F, M), dtype=torch.float32, device=A.device)
    _check(L.radar_papr(N, M, int(A.stride(1)), F, A.data_ptr(), int(A.stride(0)), out.data_ptr(),
                        _stream_ptr(stream)), "radar_papr")
    return out


def tap_wiener_weights(tap_power, noise_var_tap: float) -> list:
    """radar_tap_wiener_weights: g(n) = p(n) / (p(n) + noise_var_tap), as floats."""
    p = [float(v) for v in tap_power]
    n = len(p)
    src = (ctypes.c_double * n)(*p)
    dst = (ctypes.c_float * n)()
    _check(lib().radar_tap_wiener_weights(src, n, float(noise_var_tap), dst), "radar_tap_wiener_weights")
    return list(dst)


def workspace_bytes(cfg: Config, n_frames: int, k: int = 1) -> int:
    n = lib().radar_frame_workspace_size(ctypes.byref(cfg.desc()), int(n_frames), int(k))
    if n == 0:
        raise RadarError(RADAR_E_ARG, "radar_frame_workspace_size")
    return int(n)


def new_workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def alloc_peaks(n_frames: int, k: int, device) -> torch.Tensor:
    """Peaks buffer: int32 tensor (F, k, 5) holding radar_peak structs."""
    return torch.zeros((n_frames, k, PEAK_WORDS), dtype=torch.int32, device=device)


def unpack_peaks(peaks: torch.Tensor, n_peaks: torch.Tensor):
    """Host list (per frame) of (s, r, p, s_off, r_off) tuples."""
    pk = peaks.cpu()
    fl = pk.view(torch.float32)
    out = []
    for f in range(pk.shape[0]):
        n = int(n_peaks[f])
        out.append([(int(pk[f, i, 0]), int(pk[f, i, 1]), float(fl[f, i, 2]), float(fl[f, i, 3]),
                     float(fl[f, i, 4])) for i in range(n)])
    return out


def _check_device_buffer(x: torch.Tensor, name: str, dtype, min_elems: int, device):
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.device != device:
        raise TypeError(f"{name} must be a CUDA tensor on {device}")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if x.numel() < min_elems:
        raise ValueError(f"{name} holds {x.numel()} elements, needs at least {min_elems}")


def _check_P(P: torch.Tensor, cfg: Config, F: int, device) -> int:
    """P's frame stride in floats, after checking dtype, device, shape and row layout."""
    if not isinstance(P, torch.Tensor) or not P.is_cuda or P.device != device or P.dtype != torch.float32:
        raise TypeError(f"P must be a float32 CUDA tensor on {device}")
    shape = tuple(P.shape)
    if shape == (F, cfg.m_pad, cfg.n_pad):
        if P.stride(2) != 1 or P.stride(1) != cfg.n_pad:
            raise ValueError("P must have contiguous rows of N' floats")
        return int(P.stride(0))
    if F == 1 and shape == (cfg.m_pad, cfg.n_pad):
        if not P.is_contiguous():
            raise ValueError("P must be contiguous")
        return cfg.m_pad * cfg.n_pad
    raise ValueError(f"P must have shape ({F}, {cfg.m_pad}, {cfg.n_pad})")


def _frame_outputs(F: int, k: int, cfg: Config, dev, P, peaks, n_peaks, status, materialise: bool):
    """Allocates the outputs not given and checks those given; returns them and P's frame stride."""
    if not materialise and P is not None:
        raise ValueError("materialise=False takes no P")
    if P is None and materialise:
        P = torch.empty((F, cfg.m_pad, cfg.n_pad), dtype=torch.float32, device=dev)
    p_stride = _check_P(P, cfg, F, dev) if P is not None else 0
    if peaks is None:
        peaks = alloc_peaks(F, k, dev)
    _check_device_buffer(peaks, "peaks", torch.int32, F * k * PEAK_WORDS, dev)
    if n_peaks is None:
        n_peaks = torch.zeros(F, dtype=torch.int32, device=dev)
    _check_device_buffer(n_peaks, "n_peaks", torch.int32, F, dev)
    if status is None:
        status = torch.zeros(F, dtype=torch.int32, device=dev)
    _check_device_buffer(status, "status", torch.int32, F, dev)
    return P, p_stride, peaks, n_peaks, status


def frame_process(Y: torch.Tensor, A: torch.Tensor, cfg: Config, k: int, *, P: torch.Tensor | None = None,
                  workspace: torch.Tensor | None = None, peaks: torch.Tensor | None = None,
                  n_peaks: torch.Tensor | None = None, status: torch.Tensor | None = None, stream=None,
                  materialise: bool = True):
    """radar_frame_process on F frames: returns (P, peaks, n_peaks, status) device tensors.

    materialise=False passes P = NULL (peaks only): P is not written and None
    is returned in its place."""
    L = lib()
    Y = _as_frames(Y, cfg, "Y")
    A = _as_frames(A, cfg, "A")
    if Y.stride() != A.stride() or Y.shape != A.shape:
        raise ValueError("Y and A must share shape and strides")
    F = Y.shape[0]
    dev = Y.device
    if Y.device != A.device:
        raise ValueError("Y and A must be on one device")
    P, p_stride, peaks, n_peaks, status = _frame_outputs(F, k, cfg, dev, P, peaks, n_peaks, status, materialise)
    desc = cfg.desc(ld=Y.stride(1))
    need = workspace_bytes(cfg, F, k)
    if workspace is None or workspace.numel() < need:
        workspace = new_workspace(need, dev)
    _check_device_buffer(workspace, "workspace", torch.uint8, need, dev)
    p_ptr = P.data_ptr() if P is not None else None
    rc = L.radar_frame_process(ctypes.byref(desc), F, Y.data_ptr(), A.data_ptr(), _frame_stride(Y),
                               p_ptr, p_stride,
                               int(k), peaks.data_ptr(), n_peaks.data_ptr(), status.data_ptr(),
                               workspace.data_ptr(), workspace.numel(), _stream_ptr(stream))
    _check(rc, "radar_frame_process")
    return P, peaks, n_peaks, status


def frame_process_noalloc(Y: torch.Tensor, A: torch.Tensor, cfg: Config, k: int, *, P: torch.Tensor,
                          peaks: torch.Tensor, n_peaks: torch.Tensor, status: torch.Tensor, stream=None):
    """radar_frame_process_noalloc: radar_frame_process with the library's own
    per-device workspace (no caller workspace; nothing allocated, here or in
    the library).  Every output is the caller's; P=None means peaks only."""
    L = lib()
    Y = _as_frames(Y, cfg, "Y")
    A = _as_frames(A, cfg, "A")
    if Y.stride() != A.stride() or Y.shape != A.shape or Y.device != A.device:
        raise ValueError("Y and A must share shape, strides and device")
    F = Y.shape[0]
    for name, x in (("peaks", peaks), ("n_peaks", n_peaks), ("status", status)):
        if x is None:
            raise ValueError(f"{name} must be given")
    P, p_stride, peaks, n_peaks, status = _frame_outputs(F, k, cfg, Y.device, P, peaks, n_peaks, status,
                                                         P is not None)
    desc = cfg.desc(ld=Y.stride(1))
    rc = L.radar_frame_process_noalloc(ctypes.byref(desc), F, Y.data_ptr(), A.data_ptr(), _frame_stride(Y),
                                       P.data_ptr() if P is not None else None, p_stride, int(k),
                                       peaks.data_ptr(), n_peaks.data_ptr(), status.data_ptr(), _stream_ptr(stream))
    _check(rc, "radar_frame_process_noalloc")
    return P, peaks, n_peaks, status


def periodogram(H: torch.Tensor, cfg: Config, *, P: torch.Tensor | None = None,
                workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """radar_periodogram: Eq. 17 (with DFT-CE when n_cp < N) from an LS estimate H."""
    L = lib()
    if cfg.zc_root is not None:
        raise ValueError("radar_periodogram takes a de-precoded estimate (zc_root=None)")
    H = _as_frames(H, cfg, "H")
    F = H.shape[0]
    if P is None:
        P = torch.empty((F, cfg.m_pad, cfg.n_pad), dtype=torch.float32, device=H.device)
    need = workspace_bytes(cfg, F, 1)
    if workspace is None or workspace.numel() < need:
        workspace = new_workspace(need, H.device)
    rc = L.radar_periodogram(ctypes.byref(cfg.desc(ld=H.stride(1))), F, H.data_ptr(), _frame_stride(H),
                             P.data_ptr(), int(P.stride(0)), workspace.data_ptr(), workspace.numel(),
                             _stream_ptr(stream))
    _check(rc, "radar_periodogram")
    return P


def detect_topk(P: torch.Tensor, k: int, *, workspace: torch.Tensor | None = None, stream=None):
    """radar_detect_topk on F periodograms (F, M', N'): returns (peaks, n_peaks)."""
    L = lib()
    if not P.is_cuda or P.dtype != torch.float32:
        raise TypeError("P must be a float32 CUDA tensor")
    if P.dim() == 2:
        P = P.unsqueeze(0)
    if P.stride(2) != 1 or P.stride(1) != P.shape[2]:
        raise ValueError("P rows must be contiguous")
    F, m_pad, n_pad = P.shape
    need = L.radar_detect_workspace_size(m_pad, n_pad, F, int(k))
    if need == 0:
        raise RadarError(RADAR_E_UNSUPPORTED, "radar_detect_workspace_size")
    if workspace is None or workspace.numel() < need:
        workspace = new_workspace(need, P.device)
    peaks = alloc_peaks(F, k, P.device)
    n_peaks = torch.zeros(F, dtype=torch.int32, device=P.device)
    rc = L.radar_detect_topk(P.data_ptr(), m_pad, n_pad, F, int(P.stride(0)), int(k), peaks.data_ptr(),
                             n_peaks.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream_ptr(stream))
    _check(rc, "radar_detect_topk")
    return peaks, n_peaks


def sft_desc(k: int, dirs=None, pfa: float | None = None, tol: float | None = None) -> SftDesc:
    """radar_sft_desc with the library defaults, optionally overridden."""
    d = SftDesc()
    lib().radar_sft_default(ctypes.byref(d), int(k))
    if dirs is not None:
        if not 1 <= len(dirs) <= 16:
            raise ValueError("1 to 16 directions")
        d.n_dirs = len(dirs)
        for i, (a, b) in enumerate(dirs):
            d.dirs[i][0] = int(a)
            d.dirs[i][1] = int(b)
    if pfa is not None:
        d.pfa = float(pfa)
    if tol is not None:
        d.tol = float(tol)
    return d


def sft_workspace_bytes(cfg: Config, sft: SftDesc, n_frames: int) -> int:
    desc = cfg.desc()
    desc.flags = 0
    n = lib().radar_fps_sft_workspace_size(ctypes.byref(desc), ctypes.byref(sft), int(n_frames))
    if n == 0:
        raise RadarError(RADAR_E_ARG, "radar_fps_sft_workspace_size")
    return int(n)


def fps_sft(Y: torch.Tensor, A: torch.Tensor, cfg: Config, sft: SftDesc, *, slices: bool = False,
            workspace: torch.Tensor | None = None, stream=None):
    """radar_fps_sft on F frames: returns (peaks, n_peaks, status[, slice spectra (F, I, 3, Q)])."""
    L = lib()
    Y = _as_frames(Y, cfg, "Y")
    A = _as_frames(A, cfg, "A")
    if Y.stride() != A.stride() or Y.shape != A.shape:
        raise ValueError("Y and A must share shape and strides")
    F = Y.shape[0]
    dev = Y.device
    desc = cfg.desc(ld=Y.stride(1))
    desc.flags = 0
    peaks = alloc_peaks(F, sft.k, dev)
    n_peaks = torch.zeros(F, dtype=torch.int32, device=dev)
    status = torch.zeros(F, dtype=torch.int32, device=dev)
    S = None
    ws_ptr, ws_bytes = None, 0
    q = cfg.n_sub * cfg.n_sym // math.gcd(cfg.n_sub, cfg.n_sym)  # lcm(N, M)
    if slices:
        S = torch.empty((F, sft.n_dirs, 3, q), dtype=torch.complex64, device=dev)
    if not slices or q & (q - 1):
        # the workspace holds the spectra, and for Q not a power of two the DFT's first pass
        need = sft_workspace_bytes(cfg, sft, F)
        if workspace is None or workspace.numel() < need:
            workspace = new_workspace(need, dev)
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
    rc = L.radar_fps_sft(ctypes.byref(desc), ctypes.byref(sft), F, Y.data_ptr(), A.data_ptr(), _frame_stride(Y),
                         peaks.data_ptr(), n_peaks.data_ptr(), status.data_ptr(),
                         None if S is None else S.data_ptr(), ws_ptr, ws_bytes, _stream_ptr(stream))
    _check(rc, "radar_fps_sft")
    if slices:
        return peaks, n_peaks, status, S
    return peaks, n_peaks, status


class Batch:
    """A radar_batch plan over frames of uneven shapes.

    jobs: list of (Y, A, cfg, k) with Y, A complex64 CUDA tensors (M, N) (rows may
    be strided).  Allocates each job's P, peaks, n_peaks and status, and the
    plan's workspace; keeps references to every tensor for the plan's life.
    """

    def __init__(self, jobs, *, graph: bool = True, tune: bool = False, stream=None):
        L = lib()
        self._keep = []
        arr = (FrameJob * len(jobs))()
        self.P, self.peaks, self.n_peaks, self.status, self.k = [], [], [], [], []
        dev = None
        for i, (Y, A, cfg, k) in enumerate(jobs):
            Y = _as_frames(Y, cfg, "Y")[0]
            A = _as_frames(A, cfg, "A")[0]
            if Y.stride() != A.stride():
                raise ValueError("Y and A must share strides")
            dev = Y.device
            P = torch.empty((cfg.m_pad, cfg.n_pad), dtype=torch.float32, device=dev)
            pk = alloc_peaks(1, k, dev)[0]
            npk = torch.zeros(1, dtype=torch.int32, device=dev)
            st = torch.zeros(1, dtype=torch.int32, device=dev)
            self._keep += [Y, A]
            self.P.append(P)
            self.peaks.append(pk)
            self.n_peaks.append(npk)
            self.status.append(st)
            self.k.append(int(k))
            arr[i].d = cfg.desc(ld=Y.stride(0))
            arr[i].Y, arr[i].A, arr[i].P = Y.data_ptr(), A.data_ptr(), P.data_ptr()
            arr[i].peaks, arr[i].n_peaks, arr[i].status = pk.data_ptr(), npk.data_ptr(), st.data_ptr()
            arr[i].k = int(k)
        need = L.radar_batch_workspace_size(arr, len(jobs))
        if need == 0:
            raise RadarError(RADAR_E_ARG, "radar_batch_workspace_size")
        self.workspace = new_workspace(need, dev)
        h = ctypes.c_void_p()
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_TUNE if tune else 0)
        _check(L.radar_batch_create(arr, len(jobs), flags, self.workspace.data_ptr(), self.workspace.numel(),
                                    _stream_ptr(stream), ctypes.byref(h)), "radar_batch_create")
        self._h = h
        self._jobs = arr

    def launch(self, stream=None):
        _check(lib().radar_batch_launch(self._h, _stream_ptr(stream)), "radar_batch_launch")

    def groups(self):
        """[(n_frames, k1_mult, k3_mult, k3_generic)] per shape group."""
        L = lib()
        n = ctypes.c_int32()
        _check(L.radar_batch_info(self._h, -1, ctypes.byref(n), None, None, None, None), "radar_batch_info")
        out = []
        for g in range(n.value):
            v = [ctypes.c_int32() for _ in range(4)]
            _check(L.radar_batch_info(self._h, g, None, *[ctypes.byref(x) for x in v]), "radar_batch_info")
            out.append(tuple(x.value for x in v))
        return out

    def plans(self):
        """The tuned plan of every shape group: {n_frames, k1_mult, k3_mult,
        k3_generic, k2_half_tile, scan_groups}."""
        L = lib()
        out = []
        for g, (nf, k1, k3, gen) in enumerate(self.groups()):
            half, scan = ctypes.c_int32(), ctypes.c_int32()
            _check(L.radar_batch_plan(self._h, g, ctypes.byref(half), ctypes.byref(scan)), "radar_batch_plan")
            out.append(dict(n_frames=nf, k1_mult=k1, k3_mult=k3, k3_generic=gen, k2_half_tile=half.value,
                            scan_groups=scan.value))
        return out

    def results(self, i):
        """(P, [(s, r, p, s_off, r_off)], status) of job i (host copies)."""
        return (self.P[i].cpu().numpy(), unpack_peaks(self.peaks[i][None], self.n_peaks[i].cpu())[0],
                int(self.status[i].cpu()[0]))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().radar_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ CNN
def _f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


class CnnWorkspace:
    """Reusable device workspace of the CNN calls for batches up to `batch`."""

    def __init__(self, batch: int, train: bool, device):
        n = lib().radar_cnn_workspace_size(int(batch), int(bool(train)))
        if n == 0:
            raise RadarError(RADAR_E_ARG, "radar_cnn_workspace_size")
        self.batch, self.train = int(batch), bool(train)
        self.buf = new_workspace(n, device)


def _cnn_ws(ws, batch, train, device):
    if ws is None or ws.batch < batch or (train and not ws.train):
        ws = CnnWorkspace(batch, train, device)
    return ws


def cnn_param_count() -> int:
    return int(lib().radar_cnn_param_count())


def cnn_patches(P: torch.Tensor, peaks: torch.Tensor, n_peaks: torch.Tensor, stream=None):
    """radar_cnn_patches: P (F, M', N') float32, peaks (F, k, 5) -> (patches (F*k, 32, 32), valid (F*k,))."""
    P = _f32(P if P.dim() == 3 else P.unsqueeze(0), "P")
    F, mp, nq = P.shape
    k = peaks.shape[1]
    out = torch.empty((F * k, 32, 32), dtype=torch.float32, device=P.device)
    valid = torch.empty(F * k, dtype=torch.int32, device=P.device)
    _check(lib().radar_cnn_patches(P.data_ptr(), mp * nq, mp, nq, F, k, peaks.data_ptr(), n_peaks.data_ptr(),
                                   out.data_ptr(), valid.data_ptr(), _stream_ptr(stream)), "radar_cnn_patches")
    return out, valid


def cnn_forward(theta: torch.Tensor, patches: torch.Tensor, *, workspace: CnnWorkspace | None = None, stream=None):
    _f32(theta, "theta")
    _f32(patches, "patches")
    B = patches.shape[0]
    ws = _cnn_ws(workspace, B, False, patches.device)
    out = torch.empty((B, 2), dtype=torch.float32, device=patches.device)
    _check(lib().radar_cnn_forward(theta.data_ptr(), patches.data_ptr(), B, out.data_ptr(), ws.buf.data_ptr(),
                                   ws.buf.numel(), _stream_ptr(stream)), "radar_cnn_forward")
    return out


def cnn_gradient(theta, patches, labels, *, workspace: CnnWorkspace | None = None, stream=None):
    for t, n in ((theta, "theta"), (patches, "patches"), (labels, "labels")):
        _f32(t, n)
    B = patches.shape[0]
    ws = _cnn_ws(workspace, B, True, patches.device)
    grad = torch.empty_like(theta)
    loss = torch.empty(1, dtype=torch.float32, device=theta.device)
    _check(lib().radar_cnn_gradient(theta.data_ptr(), patches.data_ptr(), labels.data_ptr(), B, grad.data_ptr(),
                                    loss.data_ptr(), ws.buf.data_ptr(), ws.buf.numel(), _stream_ptr(stream)),
           "radar_cnn_gradient")
    return grad, loss


def cnn_adam(theta, grad, m, v, step: int, lr: float, stream=None):
    _check(lib().radar_cnn_adam(theta.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), int(step),
                                float(lr), _stream_ptr(stream)), "radar_cnn_adam")


def cnn_train_step(theta, m, v, step: int, lr: float, patches, labels, loss, *, workspace: CnnWorkspace,
                   stream=None):
    B = patches.shape[0]
    _check(lib().radar_cnn_train_step(theta.data_ptr(), m.data_ptr(), v.data_ptr(), int(step), float(lr),
                                      patches.data_ptr(), labels.data_ptr(), B, loss.data_ptr(),
                                      workspace.buf.data_ptr(), workspace.buf.numel(), _stream_ptr(stream)),
           "radar_cnn_train_step")


def timing_start(max_launches: int):
    """Start per-stage HIP-event timing inside the library (profiling aid)."""
    _check(lib().radar_timing_start(int(max_launches)), "radar_timing_start")


def timing_stop():
    """Stop stage timing; returns {stage: (total_ms, launches)}."""
    ms = (ctypes.c_double * len(STAGES))()
    cnt = (ctypes.c_int64 * len(STAGES))()
    _check(lib().radar_timing_stop(ms, cnt), "radar_timing_stop")
    return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(STAGES)}
