"""Seeded synthetic radar frames (the simulated transmitter, targets and channel).

This module is the only code shared by the oracle's tests and the GPU path's
tests and benchmark.  It draws the random quantities of one simulated frame and
applies the system model of Sec. II-B (the per-resource-element echo model that
the paper derives from Eq. 10 by dropping the time-scale and ICI terms) to
produce what the radar receives.  It holds none of the receiver's arithmetic:
no de-precoding, division, DFT-CE, window, periodogram or peak search.

Received element (symbol l, subcarrier k, both zero-based):

    y[l, k] = x_tx[l, k] * sum_p b_p exp(-j 2 pi k rho_p / N) exp(+j 2 pi l nu_p / M) + w[l, k]

* rho_p = N * delta_f * tau_p is the delay in samples (range bin),
* nu_p = M * T_s * f_D,p is the Doppler in symbol-rate bins,
* x_tx = z_k * a[l, k] is the transmitted (Zadoff-Chu precoded) symbol; the
  transmitter's precoding sequence is generated here from its definition,
* w ~ CN(0, sigma^2) with sigma^2 = 10^(-SNR/10), E|a|^2 = 1, E|b|^2 = 1.

Seeds: ``numpy.random.SeedSequence([220903883, config_id, frame_index])``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 220903883


@dataclass
class FrameSpec:
    """Everything needed to draw one frame."""

    n_sub: int                    # N subcarriers
    n_sym: int                    # M OFDM symbols
    qam: int = 4                  # 4 (QPSK) or 16
    zc_root: int | None = 1       # transmitter ZC root (None: no precoding)
    zc_shift: int = 0
    zc_dense: bool = False        # dense Z_m of a length-N^2 sequence instead of diag(z) (Eq. 24)
    n_targets: int = 3
    snr_db: float = 0.0
    on_grid: bool = True          # integer range/Doppler bins
    rho_max: float = 30.0         # range bins drawn in [rho_min, rho_max]
    rho_min: float = 1.0
    nu_abs_max: float = 31.0      # Doppler bins drawn in [-nu_abs_max, nu_abs_max]
    rayleigh: bool = False        # b ~ CN(0,1) instead of unit magnitude
    min_sep: float = 3.0          # Chebyshev separation between targets (native bins)
    noise: bool = True


@dataclass
class Frame:
    spec: FrameSpec
    Y: np.ndarray                 # (M, N) complex128, received
    A: np.ndarray                 # (M, N) complex128, data symbols known to the radar
    rho: np.ndarray               # (P,) range bins
    nu: np.ndarray                # (P,) Doppler bins
    b: np.ndarray                 # (P,) complex amplitudes
    extra: dict = field(default_factory=dict)


def rng_for(config_id: int, frame_index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, config_id, frame_index])))


def qam_symbols(rng: np.random.Generator, shape, order: int) -> np.ndarray:
    """Unit-average-power QPSK or 16-QAM symbols."""
    if order == 4:
        lv = np.array([-1.0, 1.0])
        norm = np.sqrt(2.0)
    elif order == 16:
        lv = np.array([-3.0, -1.0, 1.0, 3.0])
        norm = np.sqrt(10.0)
    else:
        raise ValueError("qam must be 4 or 16")
    re = rng.integers(0, lv.size, size=shape)
    im = rng.integers(0, lv.size, size=shape)
    return (lv[re] + 1j * lv[im]) / norm


def tx_precoding_sequence(n: int, root: int, shift: int = 0) -> np.ndarray:
    """The transmitter's length-n Zadoff-Chu sequence, written from its definition
    exp(j 2 pi r/n (k^2/2 + q k)) (even n) or exp(j 2 pi r/n (k(k+1)/2 + q k)) (odd n)."""
    k = np.arange(n, dtype=np.float64)
    quad = k * k / 2.0 if n % 2 == 0 else k * (k + 1.0) / 2.0
    return np.exp(2j * np.pi * root * (quad + shift * k) / n)


def draw_targets(rng: np.random.Generator, spec: FrameSpec):
    """Target bins with Chebyshev separation >= min_sep (by redraw)."""
    rho, nu = [], []
    tries = 0
    while len(rho) < spec.n_targets:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place targets with the requested separation")
        if spec.on_grid:
            r = float(rng.integers(int(spec.rho_min), int(spec.rho_max) + 1))
            v = float(rng.integers(-int(spec.nu_abs_max), int(spec.nu_abs_max) + 1))
        else:
            r = float(rng.uniform(spec.rho_min, spec.rho_max))
            v = float(rng.uniform(-spec.nu_abs_max, spec.nu_abs_max))
        ok = True
        for r0, v0 in zip(rho, nu):
            dv = abs(v - v0)
            dv = min(dv, spec.n_sym - dv)
            if max(abs(r - r0), dv) < spec.min_sep:
                ok = False
                break
        if ok:
            rho.append(r)
            nu.append(v)
    if spec.rayleigh:
        b = (rng.standard_normal(spec.n_targets) + 1j * rng.standard_normal(spec.n_targets)) / np.sqrt(2.0)
    else:
        b = np.exp(2j * np.pi * rng.uniform(0.0, 1.0, spec.n_targets))
    return np.array(rho), np.array(nu), b


def transmit_symbols(A: np.ndarray, spec: FrameSpec) -> np.ndarray:
    """The symbols the transmitter puts on the subcarriers: A, or A precoded
    with the spec's Zadoff-Chu sequence (diagonal), or with the N x N matrix
    Z[i, j] = zc(i N + j) of a length-N^2 sequence scaled by 1/sqrt(N) (dense)."""
    n = A.shape[-1]
    if spec.zc_root is None:
        return A
    if spec.zc_dense:
        Z = tx_precoding_sequence(n * n, spec.zc_root, spec.zc_shift).reshape(n, n)
        return A @ Z.T / np.sqrt(n)
    return A * tx_precoding_sequence(n, spec.zc_root, spec.zc_shift)[None, :]


def make_frame(spec: FrameSpec, config_id: int, frame_index: int) -> Frame:
    rng = rng_for(config_id, frame_index)
    n, m = spec.n_sub, spec.n_sym
    A = qam_symbols(rng, (m, n), spec.qam)
    rho, nu, b = draw_targets(rng, spec)
    k = np.arange(n, dtype=np.float64)
    l = np.arange(m, dtype=np.float64)
    echo = np.zeros((m, n), dtype=np.complex128)
    for p in range(spec.n_targets):
        echo += b[p] * np.outer(np.exp(2j * np.pi * l * nu[p] / m), np.exp(-2j * np.pi * k * rho[p] / n))
    tx = transmit_symbols(A, spec)
    Y = tx * echo
    if spec.noise:
        sigma2 = 10.0 ** (-spec.snr_db / 10.0)
        Y = Y + (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * np.sqrt(sigma2 / 2.0)
    return Frame(spec=spec, Y=Y, A=A, rho=rho, nu=nu, b=b)


# --------------------------------------------------------------------------
# Workload presets (shapes and value distributions of the paper's workloads)
# --------------------------------------------------------------------------
def spec_small(snr_db: float = 0.0) -> FrameSpec:
    """N=256 x M=64, QPSK, ZC root 1, three on-grid unit-magnitude targets."""
    return FrameSpec(n_sub=256, n_sym=64, qam=4, zc_root=1, n_targets=3, snr_db=snr_db,
                     on_grid=True, rho_min=1, rho_max=30, nu_abs_max=31, rayleigh=False)


def spec_full(snr_db: float = 0.0, n_sub: int = 1024, n_sym: int = 1024, n_targets: int = 8) -> FrameSpec:
    """N=1024 x M=1024 (or the 2048 x 1024 precision workload), 16-QAM, ZC root 7,
    eight off-grid Rayleigh targets inside the DFT-CE range box (range < N_cp = N/4)."""
    n_cp = n_sub // 4
    return FrameSpec(n_sub=n_sub, n_sym=n_sym, qam=16, zc_root=7, n_targets=n_targets, snr_db=snr_db,
                     on_grid=False, rho_min=1.0, rho_max=n_cp - 1.0, nu_abs_max=n_sym / 2 - 1.0,
                     rayleigh=True)


def tap_power_profile(spec: FrameSpec, grid: int = 64) -> np.ndarray:
    """E|h(n)|^2 of the generator's channel in the tap domain (the IDFT over
    the subcarriers, with 1/N), n < N: one target of delay rho gives the taps
    b D(n - rho), D(x) = (1/N) sum_k exp(2 pi i k x / N), so the profile is
    n_targets E|b|^2 E_rho |D(n - rho)|^2 over the spec's range distribution
    (integer bins, or `grid` points per bin for off-grid delays).  The
    second-order statistics a receiver with prior knowledge of the scene would
    use; separation between targets is ignored."""
    n = spec.n_sub
    if spec.on_grid:
        rhos = np.arange(int(spec.rho_min), int(spec.rho_max) + 1, dtype=np.float64)
    else:
        cnt = max(2, int(np.ceil((spec.rho_max - spec.rho_min) * grid)))
        rhos = spec.rho_min + (np.arange(cnt) + 0.5) * (spec.rho_max - spec.rho_min) / cnt
    acc = np.zeros(n)
    for c0 in range(0, rhos.size, 256):
        x = np.arange(n, dtype=np.float64)[:, None] - rhos[None, c0:c0 + 256]
        # |D(x)|^2 = sin^2(pi x) / (N^2 sin^2(pi x / N)), 1 where x is a multiple of N
        den = (n * np.sin(np.pi * x / n)) ** 2
        small = den < 1e-24
        acc += np.where(small, 1.0, np.sin(np.pi * x) ** 2 / np.where(small, 1.0, den)).sum(axis=1)
    return spec.n_targets * acc / rhos.size  # E|b|^2 = 1 (unit phasor or CN(0, 1))


def frames_to_complex64(frames):
    """Stack frames as contiguous complex64 arrays (F, M, N) for the GPU path."""
    Y = np.stack([f.Y for f in frames]).astype(np.complex64)
    A = np.stack([f.A for f in frames]).astype(np.complex64)
    return Y, A
