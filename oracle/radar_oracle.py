"""FP64 CPU oracle of the OFDM monostatic radar receive path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product path
(the HIP library and its Python binding) never imports, calls or links it, and
this module imports nothing from the product path.

Every function follows the passage of Delamou, Noubir, Dang and Amhoud, "An
Efficient OFDM-Based Monostatic Radar Design for Multitarget Detection"
(arXiv 2209.03883) that its docstring names.  The paper is a simulation study;
where it is silent, garbled or ambiguous the reading used here is stated in the
docstring and listed in the design notes.

Conventions
-----------
* All arithmetic is float64 / complex128.  numpy's FFT is used as the library
  primitive for the DFT sums; it is pinned against brute-force sums in the
  tests.
* Frames are symbol-major: ``X[l, k]`` is subcarrier ``k`` of OFDM symbol ``l``
  (the paper writes the same matrices with ``k`` as the row index).
* ``DFT_n(x)[k] = sum_i x[i] exp(-2j*pi*i*k/n)``;
  ``IDFT_n(X)[i] = (1/n) sum_k X[k] exp(+2j*pi*i*k/n)``.
"""

from __future__ import annotations

import math

import numpy as np

SPEED_OF_LIGHT = 3.0e8  # m/s, Table I

WINDOW_RECT = 0
WINDOW_HANN = 1
WINDOW_HAMMING = 2


# --------------------------------------------------------------------------
# Zadoff-Chu precoding (Sec. III-B, Eq. 23 and Eq. 24)
# --------------------------------------------------------------------------
def zc_phase_index(n: int, root: int, shift: int = 0) -> np.ndarray:
    """Exact phase indices m_k of a length-n Zadoff-Chu sequence (Eq. 23).

    Eq. 23 gives Z(k) = exp(j*2*pi*r/L * (k^2/2 + q*k)) for even L and
    exp(j*2*pi*r/L * (k(k+1)/2 + q*k)) for odd L.  Both equal
    exp(j*pi*m_k/L) with the integer
        m_k = r*(k^2 + 2qk)      mod 2L   (L even)
        m_k = r*(k(k+1) + 2qk)   mod 2L   (L odd),
    which this function returns (int64, exact).  The root r must be
    relatively prime to L (Sec. III-B); otherwise ValueError.
    """
    if n < 1:
        raise ValueError("ZC length must be positive")
    if math.gcd(int(root), int(n)) != 1:
        raise ValueError(f"ZC root {root} is not relatively prime to length {n}")
    k = np.arange(n, dtype=np.int64)
    if n % 2 == 0:
        base = k * k
    else:
        base = k * (k + 1)
    return (int(root) * ((base + 2 * int(shift) * k) % (2 * n))) % (2 * n)


def zc_sequence(n: int, root: int, shift: int = 0) -> np.ndarray:
    """Length-n Zadoff-Chu sequence z_k = exp(j*pi*m_k/n) (Eq. 23), complex128."""
    m = zc_phase_index(n, root, shift).astype(np.float64)
    ang = np.pi * m / n
    return np.cos(ang) + 1j * np.sin(ang)


ZC_DIAG = "diag"
ZC_DENSE = "dense"


def zc_matrix(n: int, root: int, shift: int = 0) -> np.ndarray:
    """The square Zadoff-Chu matrix of Eq. 24 read literally for an N-subcarrier
    symbol: a length L = N^2 sequence of Eq. 23 (root relatively prime to L)
    laid out row by row, Z_m[i, j] = Z_seq(i*N + j), D = N."""
    return zc_sequence(n * n, root, shift).reshape(n, n)


def precode_dense(A: np.ndarray, root: int, shift: int = 0) -> np.ndarray:
    """Precoded symbols A_p = Z_m A (Sec. III-B, Eq. 24 dense reading) per OFDM
    symbol, scaled by 1/sqrt(N) so that the precoding keeps the symbol energy
    (Z_m Z_m^H = N I).  A is symbol-major (M, N): row l holds symbol l, so
    A_p[l, i] = sum_j Z_m[i, j] A[l, j] / sqrt(N)."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[1]
    return A @ zc_matrix(n, root, shift).T / np.sqrt(n)


def tx_symbols(A, zc_root=None, zc_shift=0, zc_mode=ZC_DIAG):
    """The symbols the received elements carry, i.e. what the LS estimate of
    Eq. 16 divides by: A without precoding, z_k A_{l,k} under the diagonal
    reading, Z_m A / sqrt(N) under the dense one."""
    A = np.asarray(A, dtype=np.complex128)
    if zc_root is None:
        return A
    if zc_mode == ZC_DENSE:
        return precode_dense(A, zc_root, zc_shift)
    if zc_mode != ZC_DIAG:
        raise ValueError(f"unknown ZC mode {zc_mode}")
    return A * zc_sequence(A.shape[1], zc_root, zc_shift)[None, :]


# --------------------------------------------------------------------------
# Spectral division / LS channel estimate (Sec. II-B.2, Eq. 16)
# --------------------------------------------------------------------------
def ls_estimate(Y: np.ndarray, A: np.ndarray, z: np.ndarray | None = None) -> np.ndarray:
    """LS channel estimate h = y / a of Eq. 16, after ZC de-precoding.

    Sec. III-B precodes the symbols as A_p = Z_m A and removes the precoding
    at the receiver with Z_m^{-1}.  Under the diagonal reading used here
    (Z_m = diag(z_0..z_{N-1}) along the subcarriers, the same z for every
    symbol) the received element is y = z_k * a * h + noise, so
        h_{k,l} = y_{k,l} / (z_k * a_{k,l}).
    ``z=None`` means no precoding.  Zero symbols raise ZeroDivisionError.
    Under the dense reading of Eq. 24 (``tx_symbols``) the division is by the
    precoded symbols A_p themselves: applying Z_m^{-1} to the received frame
    before the division does not recover h once a target has a delay, since
    the channel multiplies each subcarrier after the precoding.
    """
    Y = np.asarray(Y, dtype=np.complex128)
    A = np.asarray(A, dtype=np.complex128)
    if Y.shape != A.shape:
        raise ValueError("Y and A must have the same shape")
    if np.any(A == 0):
        raise ZeroDivisionError("a transmitted symbol is zero")
    tx = A if z is None else A * np.asarray(z, dtype=np.complex128)[None, :]
    return Y / tx


# --------------------------------------------------------------------------
# DFT-based channel estimation (Sec. III-A, Eq. 20-22)
# --------------------------------------------------------------------------
def dft_ce(H: np.ndarray, n_cp: int) -> np.ndarray:
    """DFT-CE denoising of Sec. III-A, per OFDM symbol along the subcarriers.

    Step 1 (Eq. 20): hhat = IDFT_N(H_l), with the 1/N factor.
    Step 2 (Eq. 21): keep taps 0 <= n <= N_cp-1, zero the rest.
    Step 3 (Eq. 22): back to the frequency domain with DFT_N.  Eq. 22 prints
    a second 1/K; it is read as absent so that N_cp = N is the identity.
    """
    H = np.asarray(H, dtype=np.complex128)
    n = H.shape[1]
    if not 1 <= n_cp <= n:
        raise ValueError("n_cp must lie in [1, N]")
    taps = np.fft.ifft(H, axis=1)
    taps[:, n_cp:] = 0.0
    return np.fft.fft(taps, axis=1)


def wiener_tap_weights(tap_power, noise_var_tap: float) -> np.ndarray:
    """Per-tap LMMSE (Wiener) weights of the LMMSE-based DFT-CE of Sec. III-A
    (Fig. 5), read as a diagonal estimator in the tap domain: with the tap
    estimate hhat(n) = h(n) + w(n), E|h(n)|^2 = p(n) and white w of variance
    s per tap, the linear estimate of h(n) with least mean squared error is
    g(n) hhat(n), g(n) = p(n) / (p(n) + s)."""
    p = np.asarray(tap_power, dtype=np.float64)
    return p / (p + float(noise_var_tap))


def lmmse_dft_ce(H: np.ndarray, n_cp: int, weights) -> np.ndarray:
    """LMMSE-based DFT-CE: Eq. 20, then the kept taps n < N_cp each scaled by
    its weight (wiener_tap_weights) instead of kept whole (Eq. 21), then
    Eq. 22.  n_cp = N with the same weights is the LMMSE-based LS-CE."""
    H = np.asarray(H, dtype=np.complex128)
    g = np.asarray(weights, dtype=np.float64)
    if g.shape != (n_cp,):
        raise ValueError("one weight per kept tap")
    taps = np.fft.ifft(H, axis=1)
    taps[:, n_cp:] = 0.0
    taps[:, :n_cp] *= g[None, :]
    return np.fft.fft(taps, axis=1)


# --------------------------------------------------------------------------
# Window (Sec. II-B.2, the matrix W of Eq. 17; Hamming in Sec. IV)
# --------------------------------------------------------------------------
def window(length: int, kind: int) -> np.ndarray:
    """Periodic (DFT-even) window of the given length, float64.

    Rect: 1.  Hann: 0.5 - 0.5 cos(2 pi n / L).  Hamming: 0.54 - 0.46 cos(2 pi n / L).
    The paper does not say symmetric or periodic; the periodic form is used.
    """
    n = np.arange(length, dtype=np.float64)
    if kind == WINDOW_RECT:
        return np.ones(length)
    if kind == WINDOW_HANN:
        return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / length)
    if kind == WINDOW_HAMMING:
        return 0.54 - 0.46 * np.cos(2.0 * np.pi * n / length)
    raise ValueError(f"unknown window kind {kind}")


# --------------------------------------------------------------------------
# 2D periodogram (Sec. II-B.2, Eq. 17)
# --------------------------------------------------------------------------
def periodogram(H: np.ndarray, n_pad: int, m_pad: int, window_kind: int = WINDOW_HANN) -> np.ndarray:
    """Zero-padded, windowed 2D periodogram of Eq. 17.

        P(s, r) = 1/(N M) | sum_{k<N'} ( sum_{l<M'} h_{k,l} w_{k,l} e^{-j2pi l s/M'} ) e^{+j2pi k r/N'} |^2

    with h = 0 for k >= N or l >= M (trailing zero padding), the separable
    window w_{k,l} = w_k w_l, the printed denominators R', S' read as M', N',
    r = 0..N'-1 and the signed Doppler index s = -M'/2..M'/2-1.

    Returns float64 P with shape (M', N'); row s + M'/2 holds Doppler s.
    """
    H = np.asarray(H, dtype=np.complex128)
    m, n = H.shape
    if n_pad < n or m_pad < m:
        raise ValueError("padding must not shrink the frame")
    hw = H * window(m, window_kind)[:, None] * window(n, window_kind)[None, :]
    padded = np.zeros((m_pad, n_pad), dtype=np.complex128)
    padded[:m, :n] = hw
    doppler = np.fft.fft(padded, axis=0)            # sum over l with e^{-j...}
    rng = np.fft.ifft(doppler, axis=1) * n_pad       # sum over k with e^{+j...}
    power = (rng.real ** 2 + rng.imag ** 2) / (n * m)
    # unsigned Doppler index u -> row (u + M'/2) mod M'
    return np.roll(power, m_pad // 2, axis=0)


def frame_periodogram(Y, A, *, n_pad, m_pad, n_cp, window_kind=WINDOW_HANN,
                      zc_root=None, zc_shift=0, zc_mode=ZC_DIAG, tap_weights=None):
    """The whole estimator of Fig. 2 / Fig. 3: de-precode, divide, DFT-CE
    (LMMSE-based with per-tap weights if given), Eq. 17."""
    H = ls_estimate(Y, tx_symbols(A, zc_root, zc_shift, zc_mode))
    Hd = dft_ce(H, n_cp) if tap_weights is None else lmmse_dft_ce(H, n_cp, tap_weights)
    return periodogram(Hd, n_pad, m_pad, window_kind)


# --------------------------------------------------------------------------
# Peak extraction (Sec. II-B.2, Eq. 17-18: the dominant frequencies of P)
# --------------------------------------------------------------------------
def find_peaks(P: np.ndarray, k: int):
    """Top-k 3x3 cyclic local maxima of P.

    A cell is a peak when its value is >= each of its 8 cyclic neighbours.
    Peaks are ranked by (value descending, flat index row*N'+r ascending) and
    the first min(k, #peaks) are returned as a list of (row, r, value).
    The paper picks "the dominant peaks" of P; this is the reading used.
    """
    P = np.asarray(P)
    is_peak = np.ones(P.shape, dtype=bool)
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            if dr == 0 and dc == 0:
                continue
            is_peak &= P >= np.roll(np.roll(P, dr, axis=0), dc, axis=1)
    rows, cols = np.nonzero(is_peak)
    vals = P[rows, cols]
    flat = rows.astype(np.int64) * P.shape[1] + cols
    order = np.lexsort((flat, -vals))[:k]
    return [(int(rows[i]), int(cols[i]), float(vals[i])) for i in order]


# --------------------------------------------------------------------------
# Radar parameters (Sec. II-B.2, Eq. 13-15 and Eq. 19; Table I)
# --------------------------------------------------------------------------
def symbol_time(delta_f: float, cp_fraction: float) -> float:
    """T_s = T + T_cp with T = 1/delta_f (Sec. II-B); cp_fraction = T_cp/T."""
    return (1.0 + cp_fraction) / delta_f


def resolution(n: int, m: int, delta_f: float, f_c: float, cp_fraction: float,
               c: float = SPEED_OF_LIGHT):
    """(Delta d, Delta v) of Eq. 15."""
    ts = symbol_time(delta_f, cp_fraction)
    return c / (2.0 * n * delta_f), c / (2.0 * m * f_c * ts)


def unambiguous(delta_f: float, f_c: float, cp_fraction: float, c: float = SPEED_OF_LIGHT):
    """(d_un, v_un) of Eq. 14."""
    ts = symbol_time(delta_f, cp_fraction)
    return c / (2.0 * delta_f), c / (2.0 * f_c * ts)


def cp_max_range(delta_f: float, cp_fraction: float, c: float = SPEED_OF_LIGHT) -> float:
    """Largest range whose round trip fits the cyclic prefix (Eq. 13): c T_cp / 2."""
    return c * (cp_fraction / delta_f) / 2.0


def bins_to_range_velocity(r: float, s: float, n_pad: int, m_pad: int, delta_f: float,
                           f_c: float, cp_fraction: float, c: float = SPEED_OF_LIGHT):
    """Eq. 19 read consistently with Eq. 14-15: d = c r/(2 N' df), v = c s/(2 f_c M' T_s).

    The printed Eq. 19 swaps r and s and uses T_0 for T_s; this is the reading
    that agrees with the resolution formulas.
    """
    ts = symbol_time(delta_f, cp_fraction)
    return c * r / (2.0 * n_pad * delta_f), c * s / (2.0 * f_c * m_pad * ts)


# --------------------------------------------------------------------------
# Sub-bin refinement (Sec. II-B.2: the padded sizes N', M' "improve the
# precision" of the estimate; the refinement evaluates a 16x-padded
# periodogram locally and interpolates)
# --------------------------------------------------------------------------
FINE = 16  # the local grid is the periodogram padded 16x in both axes


def windowed_estimate(Y, A, *, n_cp, window_kind=WINDOW_HANN, zc_root=None, zc_shift=0, zc_mode=ZC_DIAG):
    """The windowed DFT-CE estimate that Eq. 17 transforms: w_k w_l H'_{l,k}."""
    n = np.asarray(Y).shape[1]
    m = np.asarray(Y).shape[0]
    Hd = dft_ce(ls_estimate(Y, tx_symbols(A, zc_root, zc_shift, zc_mode)), n_cp)
    return Hd * window(m, window_kind)[:, None] * window(n, window_kind)[None, :]


def local_periodogram(Hw: np.ndarray, sigma: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """Eq. 17 evaluated off the DFT grid, at fractional native bins.

        P(sigma, rho) = 1/(N M) | sum_l sum_k Hw[l,k] e^{-j 2 pi l sigma/M} e^{+j 2 pi k rho/N} |^2

    sigma (Doppler) and rho (range) are 1-D arrays of native-bin positions;
    returns P with shape (len(sigma), len(rho)).  At sigma = s M/M' and
    rho = r N/N' this is exactly P(s, r) of the N' x M' periodogram.
    """
    Hw = np.asarray(Hw, dtype=np.complex128)
    m, n = Hw.shape
    es = np.exp(-2j * np.pi * np.outer(np.asarray(sigma, float), np.arange(m)) / m)   # (S, M)
    er = np.exp(+2j * np.pi * np.outer(np.arange(n), np.asarray(rho, float)) / n)     # (N, R)
    G = es @ Hw @ er
    return (G.real ** 2 + G.imag ** 2) / (n * m)


def quadratic_peak_offset(F: np.ndarray):
    """Stationary point of the least-squares quadratic through a 3x3 patch.

    F[i, j] holds ln P at (x, y) = (i-1, j-1).  Fits
    a + b x + c y + d x^2 + e x y + f y^2 and solves grad = 0.  If the fitted
    Hessian is not negative definite or the point lies more than one cell
    away, falls back to the separable 3-point parabolas along x and y.
    The result is clamped to [-0.5, 0.5] per axis.
    """
    F = np.asarray(F, dtype=np.float64)
    x = np.array([-1.0, 0.0, 1.0])[:, None] * np.ones((1, 3))
    y = np.ones((3, 1)) * np.array([-1.0, 0.0, 1.0])[None, :]
    b = np.sum(x * F) / 6.0
    c = np.sum(y * F) / 6.0
    e = np.sum(x * y * F) / 4.0
    d = np.sum((x * x - 2.0 / 3.0) * F) / 2.0
    f = np.sum((y * y - 2.0 / 3.0) * F) / 2.0
    det = 4.0 * d * f - e * e
    if d < 0 and det > 0:
        ox = -(2.0 * f * b - e * c) / det
        oy = -(2.0 * d * c - e * b) / det
        if abs(ox) <= 1.0 and abs(oy) <= 1.0:
            return float(np.clip(ox, -0.5, 0.5)), float(np.clip(oy, -0.5, 0.5))

    def parabola(m1, z0, p1):
        den = m1 - 2.0 * z0 + p1
        return 0.0 if den >= 0 else float(np.clip(0.5 * (m1 - p1) / den, -0.5, 0.5))

    return parabola(F[0, 1], F[1, 1], F[2, 1]), parabola(F[1, 0], F[1, 1], F[1, 2])


def refine_peak(Hw: np.ndarray, s: int, r: int, n_pad: int, m_pad: int):
    """Sub-cell refinement of a peak at signed Doppler index s and range index r.

    The 16x-padded periodogram is evaluated on the 7 x 7 fine cells centred on
    the peak (fine cell = 1/16 native bin), the best cell of the inner 5 x 5
    is taken, and the quadratic of ln P through its 3 x 3 neighbourhood gives
    the sub-cell offset.  Returns (s_off, r_off) in cells of the N' x M' grid.
    """
    m, n = np.asarray(Hw).shape
    fs = FINE * m // m_pad          # fine cells per padded cell (Doppler)
    fr = FINE * n // n_pad          # fine cells per padded cell (range)
    cs, cr = s * fs, r * fr         # fine index of the peak
    off = np.arange(-3, 4)
    P = local_periodogram(Hw, (cs + off) / FINE, (cr + off) / FINE)
    tiny = np.finfo(np.float64).tiny
    inner = P[1:6, 1:6]
    bi, bj = np.unravel_index(np.argmax(inner), inner.shape)
    bi, bj = bi + 1, bj + 1
    patch = np.log(np.maximum(P[bi - 1:bi + 2, bj - 1:bj + 2], tiny))
    ox, oy = quadratic_peak_offset(patch)
    fine_s = (bi - 3) + ox
    fine_r = (bj - 3) + oy
    return fine_s / fs, fine_r / fr


# --------------------------------------------------------------------------
# FPS-SFT, the sparse alternative to the periodogram (Sec. III-C)
#
# The paper names the algorithm (Fourier projection-slice sparse FFT), its
# per-iteration cost (three Q-length slices, Q = lcm(N, M), one Q-point DFT
# each) and its iterative nature (components found earlier are passed on),
# and defers the rest to the algorithm's own publication.  The reading used
# here rests on the discrete projection-slice identity: for the slice
#     s_tau[t] = h[(alpha t + tau_1) mod N, (beta t + tau_2) mod M],  t < Q,
#     DFT_Q(s_tau)[m] = Q/(N M) * sum over (k1, k2) with
#                       (alpha k1 Q/N + beta k2 Q/M) = m (mod Q)
#                       of X[k1, k2] exp(+2 pi i (k1 tau_1/N + k2 tau_2/M)),
# X = DFT_N x DFT_M of h.  A bin holding one component therefore reveals k1
# and k2 through the phase ratios of the slices at offsets (1, 0) and (0, 1)
# to the slice at (0, 0).
#
# h is the LS estimate of Eq. 16 (after ZC de-precoding) indexed
# h[k, l] (subcarrier k, symbol l), without DFT-CE and without a window.
# --------------------------------------------------------------------------
# Oblique directions come first: along (1, 0) or (0, 1) every frequency of a
# range (Doppler) column lands in one bin whatever its other coordinate, so the
# bin check cannot reject a collision of two targets that share a range
# (Doppler) bin, and such collisions then decode as ghosts.
SFT_DIRECTIONS = ((1, 1), (1, -1), (1, 2), (2, 1), (1, -2), (2, -1), (1, 0), (0, 1))
SFT_OFFSETS = ((0, 0), (1, 0), (0, 1))
SFT_PFA = 1e-2     # false-alarm probability (Table I)
SFT_TOL = 0.25     # 1-sparsity tolerance on the magnitude of the slice ratios
# Bins whose power is below this fraction of the direction's largest raw bin
# power are numerically empty (rounding residue of noiseless or peeled bins).
SFT_FLOOR = 1e-10


def sft_length(n: int, m: int) -> int:
    """Q = lcm(N, M), the slice length (Sec. III-C)."""
    return n * m // math.gcd(n, m)


def sft_slices(H: np.ndarray, dirs=SFT_DIRECTIONS) -> np.ndarray:
    """The Q-point DFTs of the three slices of every direction.

    H: LS estimate [M][N] (symbol-major).  Returns S[i, j, :] = DFT_Q of the
    slice of direction dirs[i] at offset SFT_OFFSETS[j].
    """
    H = np.asarray(H, dtype=np.complex128)
    m, n = H.shape
    q = sft_length(n, m)
    t = np.arange(q, dtype=np.int64)
    S = np.empty((len(dirs), len(SFT_OFFSETS), q), dtype=np.complex128)
    for i, (a, b) in enumerate(dirs):
        for j, (t1, t2) in enumerate(SFT_OFFSETS):
            k = (a * t + t1) % n
            l = (b * t + t2) % m
            S[i, j] = np.fft.fft(H[l, k])
    return S


def sft_bin(k1: int, k2: int, a: int, b: int, n: int, m: int) -> int:
    """The bin of direction (a, b) onto which frequency (k1, k2) projects."""
    q = sft_length(n, m)
    return (a * k1 * (q // n) + b * k2 * (q // m)) % q


def sft_decode(S: np.ndarray, n: int, m: int, dirs=SFT_DIRECTIONS, k: int = 8, pfa: float = SFT_PFA,
               tol: float = SFT_TOL):
    """The iterative recovery of FPS-SFT from the slice spectra S (sft_slices).

    Directions are taken in order.  In each: the components found so far are
    peeled off the three slices; bins are visited by decreasing |S_0|
    (lower bin first on ties) down to the threshold theta, where
    theta^2 = -ln(pfa) * median(|S_0|^2) / ln 2 (the median of an exponential
    noise power is its mean times ln 2), skipping numerically empty bins
    (power below SFT_FLOOR times the largest bin power of the direction's raw
    slice, a guard that only matters without noise); a bin is taken as 1-sparse when both
    slice ratios S_1/S_0 and S_2/S_0 have magnitude within tol of 1, their
    phases decode (k1, k2), and (k1, k2) projects back onto the same bin.
    Its coefficient c = (N M / Q) S_0 is added to an already found (k1, k2) or
    starts a new component.  The search ends when k components are known or
    the directions run out.  Returns a list of [k1, k2, c].
    """
    S = np.asarray(S, dtype=np.complex128)
    q = S.shape[2]
    scale = q / (n * m)
    found: list[list] = []
    for i, (a, b) in enumerate(dirs):
        if len(found) >= k:
            break
        Si = S[i].copy()
        floor = SFT_FLOOR * float(np.max(Si[0].real ** 2 + Si[0].imag ** 2))
        for k1, k2, c in found:
            mb = sft_bin(k1, k2, a, b, n, m)
            for j, (t1, t2) in enumerate(SFT_OFFSETS):
                Si[j, mb] -= scale * c * np.exp(2j * np.pi * (k1 * t1 / n + k2 * t2 / m))
        p = Si[0].real ** 2 + Si[0].imag ** 2
        theta2 = -math.log(pfa) * float(np.median(p)) / math.log(2.0)
        for mb in np.lexsort((np.arange(q), -p)):
            if p[mb] < theta2 or p[mb] <= floor:
                break
            r1 = Si[1, mb] / Si[0, mb]
            r2 = Si[2, mb] / Si[0, mb]
            if abs(abs(r1) - 1.0) > tol or abs(abs(r2) - 1.0) > tol:
                continue
            k1 = int(np.rint(n * np.angle(r1) / (2.0 * np.pi))) % n
            k2 = int(np.rint(m * np.angle(r2) / (2.0 * np.pi))) % m
            if sft_bin(k1, k2, a, b, n, m) != mb:
                continue
            c = Si[0, mb] / scale
            for comp in found:
                if comp[0] == k1 and comp[1] == k2:
                    comp[2] += c
                    break
            else:
                found.append([k1, k2, c])
            if len(found) >= k:
                break
    return found


def sft_to_peaks(found, n: int, m: int):
    """Components as periodogram-axis detections (s, r, p), ranked like find_peaks.

    The slices use forward DFTs along both axes while Eq. 17 takes the inverse
    DFT over the subcarriers, so the range bin is r = -k1 mod N; the Doppler
    bin is k2 wrapped to [-M/2, M/2).  p = |c|^2 / (N M) is the value the
    native-resolution, rectangular-window periodogram takes at that cell.
    """
    out = []
    for k1, k2, c in found:
        s = int(k2) if k2 < m // 2 else int(k2) - m
        r = (-int(k1)) % n
        out.append((s, r, float(abs(c) ** 2 / (n * m))))
    out.sort(key=lambda e: (-e[2], (e[0] + m // 2) * n + e[1]))
    return out


def fps_sft(Y, A, *, zc_root=None, zc_shift=0, dirs=SFT_DIRECTIONS, k=8, pfa=SFT_PFA, tol=SFT_TOL):
    """FPS-SFT on one received frame: LS estimate (Eq. 16, de-precoded), slices,
    recovery; returns the detections of sft_to_peaks."""
    m, n = np.asarray(Y).shape
    z = None if zc_root is None else zc_sequence(n, zc_root, zc_shift)
    S = sft_slices(ls_estimate(Y, A, z), dirs)
    return sft_to_peaks(sft_decode(S, n, m, dirs, k, pfa, tol), n, m)


# --------------------------------------------------------------------------
# Threshold detection (Sec. II-B.2, Eq. 18)
#
# Eq. 18 declares a target where P(s, r) exceeds sigma^2 ln(P_fa); with
# ln(P_fa) < 0 the sign is garbled.  Reading: for white noise each periodogram
# cell is the squared magnitude of a circular complex Gaussian, so its power
# is exponential with mean sigma_P^2 and P(P > eta) = exp(-eta / sigma_P^2);
# the threshold for false-alarm probability P_fa is eta = -ln(P_fa) sigma_P^2.
# sigma_P^2 follows from the chain of the receiver: the LS estimate (Eq. 16)
# carries noise of variance sigma_H^2 = sigma^2 mean(1/|a|^2) per resource
# element (sigma^2 per received element); DFT-CE keeps the N_cp taps, which
# by Parseval leaves the noise power of a cell inside the cyclic-prefix range
# box unchanged; the windowed transform of Eq. 17 then gives
#     sigma_P^2 = sigma_H^2 * sum_l w_l^2 * sum_k w_k^2 / (N M).
# Detections are the local maxima of P (as find_peaks) at or above eta.
# --------------------------------------------------------------------------
def cfar_noise_power(A, noise_power: float, window_kind: int = WINDOW_HANN) -> float:
    """sigma_P^2: mean noise power of a periodogram cell (inside the CP range box)."""
    A = np.asarray(A, dtype=np.complex128)
    m, n = A.shape
    sigma_h2 = noise_power * float(np.mean(1.0 / (A.real ** 2 + A.imag ** 2)))
    wk, wl = window(n, window_kind), window(m, window_kind)
    return sigma_h2 * float(np.sum(wl * wl)) * float(np.sum(wk * wk)) / (n * m)


def cfar_threshold(A, noise_power: float, pfa: float, window_kind: int = WINDOW_HANN) -> float:
    """eta = -ln(P_fa) sigma_P^2 (Eq. 18, reading above)."""
    return -np.log(pfa) * cfar_noise_power(A, noise_power, window_kind)


def detect_threshold(P: np.ndarray, eta: float, k: int):
    """The local maxima of P at or above eta, ranked as find_peaks, at most k."""
    return [pk for pk in find_peaks(P, k) if pk[2] >= eta]


# --------------------------------------------------------------------------
# Time-domain frame simulation (Sec. II-B.1, Eq. 1-2 and Eq. 7-10)
#
# Time is counted in samples T0 = 1/(N df).  Symbol l occupies samples
# [l Ns, (l+1) Ns), Ns = N + Ng, with its cyclic prefix first; the
# transmitted waveform (Eq. 1-2) is, for t in that interval,
#     x(t) = (1/N) sum_k a_{l,k} exp(+2 pi i k (t - l Ns - Ng) / N).
# A point target p (Eq. 7-8) returns b_p exp(+2 pi i fD_p t) x(t - alpha_p(t))
# with the delay alpha_p(t) = rho_p + B_p t (rho in samples, i.e. native
# range bins).  Doppler is given in bins of the M-point Doppler DFT, so
# fD_p T0 = nu_p / (M Ns) and the per-sample CFO is eps_p = nu_p N / (M Ns)
# subcarrier spacings; the time-scale factor is B_p = fD_p / fc = eps_p df / fc.
# Reading: the time-scale term is taken at the start of each symbol's useful
# part (t_l = l Ns + Ng) and held through that symbol, so it moves the delay
# from symbol to symbol (range migration); the drift inside one symbol (B N,
# about 1e-3 samples at the paper's parameters) is dropped.  The receiver
# removes the prefix and takes the N-point DFT of each symbol's useful part.
# Eq. 11 is this model with eps_p -> 0 and B_p -> 0.
# --------------------------------------------------------------------------
def ofdm_waveform(A, n_guard: int, t) -> np.ndarray:
    """x(t) of Eq. 1-2 at (real) sample times t, zero outside the frame."""
    A = np.asarray(A, dtype=np.complex128)
    m, n = A.shape
    ns = n + n_guard
    t = np.asarray(t, dtype=np.float64)
    sym = np.floor(t / ns).astype(np.int64)
    out = np.zeros(t.shape, dtype=np.complex128)
    k = np.arange(n, dtype=np.float64)
    for i in range(t.size):
        if 0 <= sym[i] < m:
            u = t[i] - sym[i] * ns - n_guard
            out[i] = np.sum(A[sym[i]] * np.exp(2j * np.pi * k * u / n)) / n
    return out


def simulate_frame(A, targets, *, n_guard: int, fc_over_df: float, noise=None) -> np.ndarray:
    """Received frequency-domain frame Y (M, N) of the time-domain model above.

    targets: iterable of (rho, nu, b) with rho in samples, nu in Doppler bins,
    b complex.  noise: optional (M, N) added after the receiver's DFT."""
    A = np.asarray(A, dtype=np.complex128)
    m, n = A.shape
    ns = n + n_guard
    mm = np.arange(n, dtype=np.float64)
    kk = np.arange(n, dtype=np.float64)
    dft = np.exp(-2j * np.pi * np.outer(kk, mm) / n)  # receiver DFT, rows k', columns m
    Y = np.zeros((m, n), dtype=np.complex128)
    for l in range(m):
        t = l * ns + n_guard + mm                      # the useful part's sample times
        y = np.zeros(n, dtype=np.complex128)
        for rho, nu, b in targets:
            eps = nu * n / (m * ns)
            B = eps / fc_over_df
            delay = rho + B * (l * ns + n_guard)       # alpha at the symbol's start
            y += b * np.exp(2j * np.pi * nu * t / (m * ns)) * ofdm_waveform(A, n_guard, t - delay)
        Y[l] = dft @ y
    if noise is not None:
        Y = Y + np.asarray(noise, dtype=np.complex128)
    return Y


def papr(A) -> np.ndarray:
    """Peak-to-average power ratio of Eq. 25 per OFDM symbol, linear: the
    transmitted samples x_n (n < N, the N-point IDFT of the symbol's
    subcarriers; the cyclic prefix repeats samples and leaves it unchanged),
    max |x_n|^2 / mean |x_n|^2, and 0 for an all-zero symbol.  A is
    symbol-major (M, N)."""
    x = np.fft.ifft(np.asarray(A, dtype=np.complex128), axis=1)
    p = x.real ** 2 + x.imag ** 2
    mean = p.mean(axis=1)
    return np.divide(p.max(axis=1), mean, out=np.zeros_like(mean), where=mean > 0)


def hpa(A, q_db: float = 2.0) -> np.ndarray:
    """The high power amplifier of Eq. 26 applied to each symbol's transmitted
    samples, returned as the subcarrier symbols of the amplified waveform.

    Reading: an amplitude-only (AM/AM) soft limiter, the phase unchanged,
        |x'| = |x| / sqrt(1 + (|x| / (xbar 10^{q/10}))^2),
    xbar the mean of |x_n| over the symbol's N samples (the N-point IDFT; the
    prefix repeats samples), q the state level in dB (2 in Sec. III-B).  An
    all-zero symbol stays zero."""
    A = np.asarray(A, dtype=np.complex128)
    x = np.fft.ifft(A, axis=1)
    amp = np.abs(x)
    sat = amp.mean(axis=1, keepdims=True) * 10.0 ** (q_db / 10.0)
    ratio = np.divide(amp, sat, out=np.zeros_like(amp), where=sat > 0)
    return np.fft.fft(x / np.sqrt(1.0 + ratio ** 2), axis=1)
