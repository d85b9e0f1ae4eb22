"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden), closed forms, invariants, brute-force sums on tiny
inputs, and the independent channel model of the synthetic frame generator.
"""

import dataclasses
import math
import os

import numpy as np
import pytest

from oracle import radar_oracle as O
from synth import frames as S


def _load_table(path):
    rows = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows[parts[0]] = (float(parts[1]), int(parts[3]))
    return rows


# ----------------------------------------------------------------- ZC (Eq. 23)
def test_zc_worked_example(golden_dir):
    data = np.loadtxt(os.path.join(golden_dir, "zc_n4_root1.txt"))
    m = O.zc_phase_index(4, 1)
    z = O.zc_sequence(4, 1)
    np.testing.assert_array_equal(m, data[:, 1].astype(np.int64))
    np.testing.assert_allclose(z.real, data[:, 2], atol=1e-15)
    np.testing.assert_allclose(z.imag, data[:, 3], atol=1e-15)
    # lag-1 cyclic autocorrelation of this sequence is zero
    assert abs(np.sum(z * np.conj(np.roll(z, 1)))) < 1e-15


@pytest.mark.parametrize("n,root", [(256, 1), (1024, 7), (2048, 7), (255, 2), (63, 5), (7, 3)])
def test_zc_cazac(n, root):
    z = O.zc_sequence(n, root)
    np.testing.assert_allclose(np.abs(z), 1.0, atol=1e-14)
    # periodic autocorrelation: N at lag 0, zero elsewhere (CAZAC, Sec. III-B)
    ac = np.fft.ifft(np.abs(np.fft.fft(z)) ** 2) * 1.0
    assert abs(ac[0] - n) < 1e-9 * n
    assert np.max(np.abs(ac[1:])) < 1e-12 * n
    # flat spectrum |DFT(z)| = sqrt(N)
    np.testing.assert_allclose(np.abs(np.fft.fft(z)), math.sqrt(n), rtol=1e-11)


def test_zc_phase_matches_definition_brute_force():
    # Eq. 23 evaluated term by term in exact rational arithmetic of the phase.
    for n, root, q in [(8, 3, 0), (8, 5, 2), (9, 2, 1), (16, 7, 3)]:
        m = O.zc_phase_index(n, root, q)
        for k in range(n):
            if n % 2 == 0:
                num = root * (k * k + 2 * q * k)       # 2*pi*r/L*(k^2/2+qk) = pi*num/L
            else:
                num = root * (k * (k + 1) + 2 * q * k)
            assert (num - int(m[k])) % (2 * n) == 0


def test_zc_root_must_be_coprime():
    with pytest.raises(ValueError):
        O.zc_phase_index(1024, 2)
    with pytest.raises(ValueError):
        O.zc_phase_index(9, 3)


# ------------------------------------------- dense ZC matrix (Eq. 24, literal)
def test_zc_matrix_worked_example(golden_dir):
    data = np.loadtxt(os.path.join(golden_dir, "zc_matrix_n2_root1.txt"))
    Z = O.zc_matrix(2, 1)
    for i, j, re, im in data:
        assert Z[int(i), int(j)] == pytest.approx(complex(re, im), abs=1e-15)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 9, 15, 16, 64, 256])
def test_zc_matrix_rows_orthogonal(n):
    # Z_m Z_m^H = N I for every root prime to N and any shift
    for root in (1, 3, 5, 7):
        if math.gcd(root, n) != 1:
            continue
        for q in (0, 3):
            Z = O.zc_matrix(n, root, q)
            np.testing.assert_allclose(Z @ Z.conj().T, n * np.eye(n), atol=1e-12 * n)


@pytest.mark.parametrize("n,root,q", [(8, 3, 0), (16, 5, 2), (64, 7, 1), (256, 1, 0), (1024, 7, 0)])
def test_zc_matrix_factorisation(n, root, q):
    # (iN + j)^2 = i^2 N^2 + 2ijN + j^2 splits Eq. 24 for even N into
    # Z_m = D1 F D2: D1(i) = e^{j pi r (i^2 + 2qi/N)}, F(i, j) = e^{j 2 pi r ij/N},
    # D2(j) = e^{j pi r (j^2 + 2qj)/N^2}; an N-point DFT between two diagonals
    i = np.arange(n)
    d1 = np.exp(1j * np.pi * ((root * (i * i + 2 * q * i / n)) % 2))
    d2 = np.exp(1j * np.pi * root * ((i * i + 2 * q * i) % (2 * n * n)) / (n * n))
    F = np.exp(2j * np.pi * ((root * np.outer(i, i)) % n) / n)
    np.testing.assert_allclose(O.zc_matrix(n, root, q), d1[:, None] * F * d2[None, :], atol=1e-9)


def test_dense_precoding_keeps_symbol_energy():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((5, 64)) + 1j * rng.standard_normal((5, 64))
    Ap = O.precode_dense(A, 3, 1)
    np.testing.assert_allclose(np.sum(np.abs(Ap) ** 2, axis=1), np.sum(np.abs(A) ** 2, axis=1), rtol=1e-12)
    # symbol by symbol, and the literal matrix-vector product
    Z = O.zc_matrix(64, 3, 1)
    np.testing.assert_allclose(Ap[2], Z @ A[2] / 8.0, atol=1e-12)


def test_dense_precoding_recovers_generator_channel():
    spec = S.FrameSpec(n_sub=64, n_sym=16, qam=16, zc_root=5, zc_shift=2, zc_dense=True, n_targets=2,
                       noise=False, on_grid=False, rho_max=14, nu_abs_max=7, rayleigh=True)
    f = S.make_frame(spec, 99, 0)
    H = O.ls_estimate(f.Y, O.tx_symbols(f.A, 5, 2, O.ZC_DENSE))
    k = np.arange(64)
    l = np.arange(16)
    ref = sum(f.b[p] * np.outer(np.exp(2j * np.pi * l * f.nu[p] / 16), np.exp(-2j * np.pi * k * f.rho[p] / 64))
              for p in range(2))
    np.testing.assert_allclose(H, ref, atol=1e-9)
    # de-precoding the received frame with Z_m^{-1} first, then dividing by A,
    # does not give the channel (the reading that Eq. 24's inverse cannot take)
    Zinv = np.linalg.inv(O.zc_matrix(64, 5, 2) / 8.0)
    H_lit = (f.Y @ Zinv.T) / f.A
    assert np.max(np.abs(H_lit - ref)) > 0.1


def test_dense_precoding_periodogram_single_target():
    # noiseless: the LS estimate is the channel itself, so P is the precoding-free P
    kw = dict(n_sub=128, n_sym=32, qam=16, zc_root=7, n_targets=1, noise=False, rho_max=20, nu_abs_max=10)
    fd = S.make_frame(S.FrameSpec(zc_dense=True, **kw), 5, 0)
    fn = S.make_frame(S.FrameSpec(**{**kw, "zc_root": None}), 5, 0)
    Pd = O.frame_periodogram(fd.Y, fd.A, n_pad=512, m_pad=128, n_cp=32, zc_root=7, zc_mode=O.ZC_DENSE)
    Pn = O.frame_periodogram(fn.Y, fn.A, n_pad=512, m_pad=128, n_cp=32)
    np.testing.assert_allclose(Pd, Pn, atol=1e-9 * Pn.max())


# ------------------------------------------- LMMSE-based DFT-CE (Fig. 5)
@pytest.mark.parametrize("p,s", [(1.0, 1.0), (4.0, 0.5), (0.1, 2.0), (1e-3, 1e-3)])
def test_wiener_weight_mse_closed_form(p, s):
    # h ~ CN(0, p), hhat = h + w, w ~ CN(0, s): E|g hhat - h|^2 = p s / (p + s),
    # below both the raw estimate's s and the zero estimate's p
    rng = np.random.default_rng(7)
    n = 400000
    h = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * np.sqrt(p / 2)
    x = h + (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * np.sqrt(s / 2)
    g = float(O.wiener_tap_weights([p], s)[0])
    mse = float(np.mean(np.abs(g * x - h) ** 2))
    assert mse == pytest.approx(p * s / (p + s), rel=0.02)
    assert mse < min(p, s)
    # and g is the minimiser: nudging it either way costs
    assert mse < float(np.mean(np.abs(1.05 * g * x - h) ** 2)) and mse < float(np.mean(np.abs(0.95 * g * x - h) ** 2))


def test_lmmse_dft_ce_unit_weights_is_dft_ce():
    rng = np.random.default_rng(8)
    H = rng.standard_normal((4, 64)) + 1j * rng.standard_normal((4, 64))
    np.testing.assert_allclose(O.lmmse_dft_ce(H, 16, np.ones(16)), O.dft_ce(H, 16), atol=1e-13)
    # weights far above the noise tend to 1; zero prior power removes the tap
    g = O.wiener_tap_weights(np.r_[np.full(8, 1e12), np.zeros(8)], 1.0)
    np.testing.assert_allclose(g, np.r_[np.ones(8), np.zeros(8)], atol=1e-11)


def test_tap_power_profile():
    on = S.FrameSpec(n_sub=64, n_sym=8, n_targets=3, on_grid=True, rho_min=2, rho_max=9)
    p = S.tap_power_profile(on)
    np.testing.assert_allclose(p[2:10], 3 / 8, rtol=1e-12)
    assert np.max(np.abs(np.r_[p[:2], p[10:]])) < 1e-12
    off = S.FrameSpec(n_sub=128, n_sym=8, n_targets=5, on_grid=False, rho_min=1.0, rho_max=20.0)
    q = S.tap_power_profile(off)
    assert float(q.sum()) == pytest.approx(5.0, rel=1e-9)  # Parseval: each target brings unit energy
    # one delay, brute force: taps of exp(-2 pi i k rho / N) by the IDFT sum
    k = np.arange(128)
    taps = np.array([np.mean(np.exp(-2j * np.pi * k * 7.3 / 128) * np.exp(2j * np.pi * k * n / 128))
                     for n in range(128)])
    one = S.tap_power_profile(dataclasses.replace(off, n_targets=1, rho_min=7.3, rho_max=7.3 + 1e-9), grid=1)
    np.testing.assert_allclose(one, np.abs(taps) ** 2, atol=1e-9)


def test_lmmse_estimators_mse_ordering():
    # Fig. 5: channel MSE of LMMSE-based DFT-CE < DFT-CE < LS-CE, and
    # LMMSE-based LS-CE < LS-CE, on the generator's frames with its own prior
    spec = S.FrameSpec(n_sub=256, n_sym=32, qam=16, zc_root=3, n_targets=4, snr_db=-5.0, on_grid=False,
                       rho_min=1.0, rho_max=40.0, nu_abs_max=15.0, rayleigh=True)
    n_cp = 64
    prior = S.tap_power_profile(spec)
    sigma2 = 10 ** (5.0 / 10)
    err = {"ls": 0.0, "lmmse_ls": 0.0, "dft": 0.0, "lmmse_dft": 0.0}
    for i in range(6):
        f = S.make_frame(spec, 90, i)
        H = O.ls_estimate(f.Y, O.tx_symbols(f.A, 3))
        k, l = np.arange(256), np.arange(32)
        true = sum(f.b[p] * np.outer(np.exp(2j * np.pi * l * f.nu[p] / 32), np.exp(-2j * np.pi * k * f.rho[p] / 256))
                   for p in range(spec.n_targets))
        s_tap = sigma2 * float(np.mean(1.0 / np.abs(f.A) ** 2)) / 256
        est = {"ls": H, "dft": O.dft_ce(H, n_cp),
               "lmmse_ls": O.lmmse_dft_ce(H, 256, O.wiener_tap_weights(prior, s_tap)),
               "lmmse_dft": O.lmmse_dft_ce(H, n_cp, O.wiener_tap_weights(prior[:n_cp], s_tap))}
        for key, v in est.items():
            err[key] += float(np.mean(np.abs(v - true) ** 2))
    assert err["lmmse_dft"] < err["dft"] < err["ls"]
    assert err["lmmse_ls"] < err["ls"]


# ---------------------------------------------------------------- HPA (Eq. 26)
def test_hpa_closed_forms():
    n = 64
    rng = np.random.default_rng(24)
    # one subcarrier: a constant envelope |x| = xbar, so every sample is scaled
    # by 1 / sqrt(1 + 10^{-q/5})
    one = np.zeros((2, n), complex)
    one[0, 9] = 1.5 - 0.5j
    for q in (0.0, 2.0, 6.0):
        np.testing.assert_allclose(O.hpa(one, q)[0], one[0] / np.sqrt(1.0 + 10.0 ** (-q / 5.0)), atol=1e-13)
    assert np.all(O.hpa(one, 2.0)[1] == 0)  # nothing sent, nothing amplified
    # far below saturation: linear
    A = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    np.testing.assert_allclose(O.hpa(A, 200.0), A, atol=1e-9)
    # the output envelope stays below the saturation level, the phase is kept
    x = np.fft.ifft(A, axis=1)
    y = np.fft.ifft(O.hpa(A, 2.0), axis=1)
    sat = np.abs(x).mean(axis=1, keepdims=True) * 10 ** 0.2
    assert np.all(np.abs(y) < sat)
    np.testing.assert_allclose(np.angle(y * np.conj(x)), 0.0, atol=1e-9)
    # brute force, sample by sample
    k = np.arange(n)
    for l in range(3):
        xs = np.array([np.sum(A[l] * np.exp(2j * np.pi * k * m / n)) / n for m in range(n)])
        s = np.mean(np.abs(xs)) * 10 ** 0.2
        ys = xs / np.sqrt(1 + (np.abs(xs) / s) ** 2)
        ref = np.array([np.sum(ys * np.exp(-2j * np.pi * np.arange(n) * kk / n)) for kk in range(n)])
        np.testing.assert_allclose(O.hpa(A, 2.0)[l], ref, atol=1e-10)


# ----------------------------------- time-domain frame model (Eq. 1-2, 7-10)
def _qpsk(rng, m, n):
    return (rng.choice([-1.0, 1.0], (m, n)) + 1j * rng.choice([-1.0, 1.0], (m, n))) / np.sqrt(2.0)


def test_time_domain_static_target_is_eq11():
    # no motion, delay inside the prefix: the received symbol is a times the
    # channel's phase ramp, exactly (Eq. 11 holds with equality)
    rng = np.random.default_rng(21)
    A = _qpsk(rng, 8, 32)
    for rho in (0.0, 3.0, 5.5, 8.0):
        Y = O.simulate_frame(A, [(rho, 0.0, 0.7 - 0.2j)], n_guard=8, fc_over_df=320833.0)
        k = np.arange(32)
        np.testing.assert_allclose(Y, (0.7 - 0.2j) * A * np.exp(-2j * np.pi * k * rho / 32)[None, :], atol=1e-12)


def test_time_domain_ici_closed_form():
    # one active subcarrier k0, Doppler eps subcarrier spacings: the receiver
    # sees |D(eps - q)| at k0 + q, D(x) = sin(pi x) / (N sin(pi x / N))
    m, n, ng = 4, 64, 16
    A = np.zeros((m, n), complex)
    k0 = 20
    A[:, k0] = 1.0
    for nu in (0.3, 1.7, -2.2):
        eps = nu * n / (m * (n + ng))
        Y = O.simulate_frame(A, [(2.0, nu, 1.0)], n_guard=ng, fc_over_df=320833.0)
        for q in range(-3, 4):
            x = eps - q
            ref = abs(np.sin(np.pi * x) / (n * np.sin(np.pi * x / n)))
            assert abs(Y[1, k0 + q]) == pytest.approx(ref, rel=1e-9, abs=1e-13)


def test_time_domain_range_migration_phase():
    # the time-scale factor moves the delay by B (l Ns + Ng) from symbol to
    # symbol: the phase of one subcarrier follows it (a small fc/df makes the
    # effect large)
    m, n, ng, fc_df, nu, rho = 6, 32, 8, 40.0, 1.5, 2.0
    A = np.zeros((m, n), complex)
    k0 = 9
    A[:, k0] = 1.0
    Y = O.simulate_frame(A, [(rho, nu, 1.0)], n_guard=ng, fc_over_df=fc_df)
    ns = n + ng
    eps = nu * n / (m * ns)
    B = eps / fc_df
    dsum = np.sum(np.exp(2j * np.pi * eps * np.arange(n) / n)) / n
    for l in range(m):
        tl = l * ns + ng
        ref = np.exp(2j * np.pi * nu * tl / (m * ns)) * np.exp(-2j * np.pi * k0 * (rho + B * tl) / n) * dsum
        assert Y[l, k0] == pytest.approx(ref, abs=1e-12)


def test_time_domain_slow_targets_approach_eq11():
    # as the Doppler shrinks, the frame approaches Eq. 11 (the generator's
    # frequency-domain model) up to the constant phase of the prefix
    rng = np.random.default_rng(22)
    m, n, ng = 16, 64, 16
    A = _qpsk(rng, m, n)
    k, l = np.arange(n), np.arange(m)
    errs = []
    for nu in (2.0, 0.2, 0.02):
        Y = O.simulate_frame(A, [(4.0, nu, 1.0)], n_guard=ng, fc_over_df=320833.0)
        eq11 = A * np.outer(np.exp(2j * np.pi * l * nu / m), np.exp(-2j * np.pi * k * 4.0 / n))
        eq11 *= np.exp(2j * np.pi * nu * ng / (m * (n + ng)))
        errs.append(float(np.max(np.abs(Y - eq11))))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.01


# --------------------------------------------------------------- PAPR (Eq. 25)
def test_papr_closed_forms():
    n = 64
    one = np.zeros((1, n), complex)
    one[0, 5] = 2.0 - 1.0j
    assert O.papr(one)[0] == pytest.approx(1.0, abs=1e-12)      # one subcarrier: constant envelope
    assert O.papr(np.ones((1, n), complex))[0] == pytest.approx(n, rel=1e-12)  # all in phase: an impulse
    assert O.papr(np.zeros((1, n), complex))[0] == 0.0                         # nothing sent
    # a brute-force IDFT for random symbols, and the bound PAPR <= N
    rng = np.random.default_rng(23)
    A = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    k = np.arange(n)
    for l in range(3):
        x = np.array([np.sum(A[l] * np.exp(2j * np.pi * k * m / n)) for m in range(n)]) / n
        p = np.abs(x) ** 2
        assert O.papr(A)[l] == pytest.approx(p.max() / p.mean(), rel=1e-12)
    assert np.all(O.papr(A) <= n + 1e-9)


# ------------------------------------------------------- division (Eq. 16)
def test_ls_estimate_recovers_generator_channel():
    spec = S.FrameSpec(n_sub=64, n_sym=16, qam=16, zc_root=5, n_targets=2, noise=False,
                       on_grid=False, rho_max=14, nu_abs_max=7, rayleigh=True)
    f = S.make_frame(spec, 99, 0)
    H = O.ls_estimate(f.Y, f.A, O.zc_sequence(64, 5))
    k = np.arange(64)
    l = np.arange(16)
    ref = sum(f.b[p] * np.outer(np.exp(2j * np.pi * l * f.nu[p] / 16), np.exp(-2j * np.pi * k * f.rho[p] / 64))
              for p in range(2))
    np.testing.assert_allclose(H, ref, atol=1e-13)


def test_ls_estimate_rejects_zero_symbol():
    A = np.ones((2, 4), complex)
    A[1, 2] = 0
    with pytest.raises(ZeroDivisionError):
        O.ls_estimate(np.ones((2, 4), complex), A)


# -------------------------------------------------------- DFT-CE (Eq. 20-22)
def test_dft_ce_identity_and_projection():
    rng = np.random.default_rng(1)
    H = rng.standard_normal((6, 32)) + 1j * rng.standard_normal((6, 32))
    np.testing.assert_allclose(O.dft_ce(H, 32), H, atol=1e-13)
    D = O.dft_ce(H, 8)
    np.testing.assert_allclose(O.dft_ce(D, 8), D, atol=1e-13)       # idempotent
    assert np.sum(np.abs(D) ** 2) <= np.sum(np.abs(H) ** 2) + 1e-9  # energy never grows
    # orthogonal projection: residual is orthogonal to the kept part
    assert abs(np.vdot(D, H - D)) < 1e-9


def test_dft_ce_brute_force_tiny():
    rng = np.random.default_rng(2)
    n, n_cp = 8, 3
    H = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    out = O.dft_ce(H, n_cp)
    for l in range(2):
        taps = [sum(H[l, k] * np.exp(2j * np.pi * i * k / n) for k in range(n)) / n for i in range(n)]
        for k in range(n):
            ref = sum(taps[i] * np.exp(-2j * np.pi * i * k / n) for i in range(n_cp))
            assert abs(out[l, k] - ref) < 1e-12


def test_dft_ce_passes_target_inside_cp():
    n, m = 64, 8
    k = np.arange(n)
    l = np.arange(m)
    H = 0.7 * np.outer(np.exp(2j * np.pi * l * 3 / m), np.exp(-2j * np.pi * k * 11 / n))
    np.testing.assert_allclose(O.dft_ce(H, 16), H, atol=1e-13)
    # and removes one outside it
    H2 = np.outer(np.ones(m), np.exp(-2j * np.pi * k * 40 / n))
    assert np.max(np.abs(O.dft_ce(H2, 16))) < 1e-13


def test_dft_ce_white_noise_energy_fraction():
    rng = np.random.default_rng(3)
    n, n_cp = 256, 64
    W = (rng.standard_normal((400, n)) + 1j * rng.standard_normal((400, n))) / np.sqrt(2)
    ratio = np.sum(np.abs(O.dft_ce(W, n_cp)) ** 2) / np.sum(np.abs(W) ** 2)
    # ratio is a mean of 400*256 chi-square terms: expected n_cp/n, sd ~ 0.25/sqrt(400*64)
    assert abs(ratio - n_cp / n) < 0.01


# ----------------------------------------------------------- window
def test_windows_periodic():
    w = O.window(8, O.WINDOW_HANN)
    np.testing.assert_allclose(w, [0, 0.14644660940672624, 0.5, 0.8535533905932737, 1.0,
                                   0.8535533905932737, 0.5, 0.14644660940672624], atol=1e-15)
    assert abs(O.window(64, O.WINDOW_HANN).sum() - 32) < 1e-12
    assert abs(O.window(64, O.WINDOW_HAMMING).sum() - 0.54 * 64) < 1e-12
    np.testing.assert_array_equal(O.window(5, O.WINDOW_RECT), np.ones(5))


# --------------------------------------------------------- periodogram (Eq. 17)
def _periodogram_brute(H, n_pad, m_pad, wk):
    m, n = H.shape
    w_l = O.window(m, wk)
    w_k = O.window(n, wk)
    P = np.zeros((m_pad, n_pad))
    for s in range(-m_pad // 2, m_pad // 2):
        for r in range(n_pad):
            acc = 0j
            for k in range(n):
                inner = 0j
                for l in range(m):
                    inner += H[l, k] * w_k[k] * w_l[l] * np.exp(-2j * np.pi * l * s / m_pad)
                acc += inner * np.exp(2j * np.pi * k * r / n_pad)
            P[s + m_pad // 2, r] = abs(acc) ** 2 / (n * m)
    return P


@pytest.mark.parametrize("wk", [O.WINDOW_RECT, O.WINDOW_HANN, O.WINDOW_HAMMING])
def test_periodogram_brute_force_tiny(wk):
    rng = np.random.default_rng(4 + wk)
    H = rng.standard_normal((4, 8)) + 1j * rng.standard_normal((4, 8))
    P = O.periodogram(H, 32, 16, wk)
    ref = _periodogram_brute(H, 32, 16, wk)
    assert np.max(np.abs(P - ref)) < 1e-12 * np.max(ref)


@pytest.mark.parametrize("wk,gain", [(O.WINDOW_RECT, 1.0), (O.WINDOW_HANN, 0.5), (O.WINDOW_HAMMING, 0.54)])
def test_periodogram_single_target_closed_form(wk, gain):
    n, m, n_pad, m_pad = 64, 32, 256, 128
    rho, nu, b = 13, -5, 0.8 * np.exp(0.3j)
    k = np.arange(n)
    l = np.arange(m)
    H = b * np.outer(np.exp(2j * np.pi * l * nu / m), np.exp(-2j * np.pi * k * rho / n))
    P = O.periodogram(H, n_pad, m_pad, wk)
    row, col = np.unravel_index(np.argmax(P), P.shape)
    assert (row - m_pad // 2, col) == (nu * m_pad // m, rho * n_pad // n)
    # P = |b|^2 (sum w_k)^2 (sum w_l)^2 / (N M) = |b|^2 g^4 N M
    assert abs(P[row, col] - abs(b) ** 2 * gain ** 4 * n * m) < 1e-9 * P[row, col]


def test_periodogram_parseval():
    rng = np.random.default_rng(5)
    H = rng.standard_normal((16, 32)) + 1j * rng.standard_normal((16, 32))
    P = O.periodogram(H, 128, 64, O.WINDOW_HANN)
    hw = H * O.window(16, 1)[:, None] * O.window(32, 1)[None, :]
    assert abs(P.sum() - (128 * 64) / (32 * 16) * np.sum(np.abs(hw) ** 2)) < 1e-9 * P.sum()


@pytest.mark.parametrize("wk", [O.WINDOW_HANN, O.WINDOW_HAMMING])
def test_periodogram_dftce_zero_pattern(wk):
    # After DFT-CE the taps live on [0, N_cp); a cosine window widens them to
    # [-1, N_cp]; at N' = 4N the range samples r = 4q are those taps scaled,
    # so P[:, 4q] vanishes for q in [N_cp+1, N-2].
    rng = np.random.default_rng(6)
    n, m, n_cp = 64, 16, 16
    H = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    P = O.periodogram(O.dft_ce(H, n_cp), 4 * n, 2 * m, wk)
    zero_cols = [4 * q for q in range(n_cp + 1, n - 1)]
    assert np.max(P[:, zero_cols]) < 1e-13 * np.max(P)
    assert np.min(np.max(P[:, [4 * q for q in range(0, n_cp)]], axis=0)) > 1e-6 * np.max(P)


def test_frame_periodogram_finds_generator_targets():
    f = S.make_frame(S.spec_small(snr_db=10.0), 1, 0)
    P = O.frame_periodogram(f.Y, f.A, n_pad=1024, m_pad=256, n_cp=32, zc_root=1)
    got = sorted((r - 128, c) for r, c, _ in O.find_peaks(P, 3))
    want = sorted((int(v * 4), int(r * 4)) for r, v in zip(f.rho, f.nu))
    assert got == want


# ---------------------------------------------------------------- peaks
def _peaks_brute(P, k):
    R, C = P.shape
    found = []
    for i in range(R):
        for j in range(C):
            ok = True
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    if (di or dj) and P[(i + di) % R, (j + dj) % C] > P[i, j]:
                        ok = False
            if ok:
                found.append((-P[i, j], i * C + j, i, j))
    found.sort()
    return [(i, j, -v) for v, _, i, j in found[:k]]


def test_find_peaks_brute_force_with_ties_and_wrap():
    rng = np.random.default_rng(7)
    for trial in range(20):
        P = np.round(rng.random((9, 12)) * 6) / 6      # many exact ties
        P[0, 0] = 2.0                                   # corner peak, wraps both ways
        P[8, 11] = 2.0                                  # its diagonal neighbour: a tie
        P[4, 11] = 1.5                                  # wraps along columns
        assert O.find_peaks(P, 10) == _peaks_brute(P, 10)


def test_find_peaks_returns_fewer_when_few_peaks():
    # a single cyclic "hill": every other cell has a strictly larger neighbour
    i, j = np.meshgrid(np.arange(6), np.arange(8), indexing="ij")
    di = np.minimum(np.abs(i - 1), 6 - np.abs(i - 1))
    dj = np.minimum(np.abs(j - 2), 8 - np.abs(j - 2))
    P = 10.0 - di - dj
    assert O.find_peaks(P, 5) == [(1, 2, 10.0)]
    # a flat plateau: every cell is >= its neighbours, so all are peaks,
    # ranked by flat index
    assert O.find_peaks(np.zeros((3, 3)), 4) == [(0, 0, 0.0), (0, 1, 0.0), (0, 2, 0.0), (1, 0, 0.0)]


# ------------------------------------------------------- Table I numbers
def test_table1_derived_numbers(golden_dir):
    t = _load_table(os.path.join(golden_dir, "table1_parameters.txt"))
    n, m = int(t["n_sub"][0]), int(t["n_sym"][0])
    df, fc, cpf = t["delta_f"][0], t["f_c"][0], t["cp_fraction"][0]

    def printed(name, value, scale=1.0):
        want, dec = t[name]
        assert round(value * scale, dec) == pytest.approx(want, abs=10 ** -(dec + 3)), name

    dd, dv = O.resolution(n, m, df, fc, cpf)
    printed("range_resolution_cm", dd, 100.0)
    printed("velocity_resolution_cms", dv, 100.0)
    printed("velocity_resolution", dv)
    printed("max_range", O.cp_max_range(df, cpf))
    assert n * df == t["bandwidth"][0]
    d_un, v_un = O.unambiguous(df, fc, cpf)
    assert d_un == pytest.approx(625.0)
    assert v_un == pytest.approx(374.03, abs=5e-3)
    assert dd == pytest.approx(d_un / n) and dv == pytest.approx(v_un / m)
    # Sec. IV prints 43.73 m for the 7 % normal CP; c*0.07/(2*240 kHz) = 43.75 m.
    assert abs(O.cp_max_range(df, t["normal_cp_fraction"][0]) - t["normal_cp_max_range"][0]) < 0.03


def test_bins_to_units():
    # one native bin maps to one resolution cell (Eq. 15 vs Eq. 19)
    d, v = O.bins_to_range_velocity(4.0, 4.0, 4 * 2048, 4 * 560, 240e3, 77e9, 0.25)
    dd, dv = O.resolution(2048, 560, 240e3, 77e9, 0.25)
    assert d == pytest.approx(dd) and v == pytest.approx(dv)


# ------------------------------------------------- sub-cell refinement
def test_local_periodogram_on_grid_equals_padded_fft():
    # At sigma = s M/M', rho = r N/N' the off-grid sum is the N' x M'
    # periodogram of Eq. 17 (FFT route, pinned by brute force above).
    rng = np.random.default_rng(21)
    m, n, mp, nq = 16, 32, 64, 128
    H = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    Hd = O.dft_ce(H, 8)
    Pfft = O.periodogram(Hd, nq, mp, O.WINDOW_HANN)
    Hw = Hd * O.window(m, O.WINDOW_HANN)[:, None] * O.window(n, O.WINDOW_HANN)[None, :]
    s = np.arange(-mp // 2, mp // 2)
    r = np.arange(nq)
    Ploc = O.local_periodogram(Hw, s * m / mp, r * n / nq)
    np.testing.assert_allclose(Ploc, Pfft, rtol=1e-10, atol=1e-12 * Pfft.max())


def test_local_periodogram_brute_force_off_grid():
    rng = np.random.default_rng(22)
    m, n = 3, 5
    Hw = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    sig, rho = [0.3, -1.7], [2.25, 0.0, 4.9]
    got = O.local_periodogram(Hw, sig, rho)
    for a, sv in enumerate(sig):
        for b_, rv in enumerate(rho):
            g = 0j
            for l in range(m):
                for k in range(n):
                    g += Hw[l, k] * complex(math.cos(-2 * math.pi * l * sv / m), math.sin(-2 * math.pi * l * sv / m)) \
                        * complex(math.cos(2 * math.pi * k * rv / n), math.sin(2 * math.pi * k * rv / n))
            assert got[a, b_] == pytest.approx(abs(g) ** 2 / (n * m), rel=1e-12)


def _quad_patch(x0, y0, hxx, hxy, hyy, a=1.0):
    x = np.array([-1.0, 0.0, 1.0])[:, None]
    y = np.array([-1.0, 0.0, 1.0])[None, :]
    dx, dy = x - x0, y - y0
    return a + 0.5 * (hxx * dx * dx + 2 * hxy * dx * dy + hyy * dy * dy)


def test_quadratic_offset_exact_on_quadratics():
    # a concave quadratic is its own least-squares fit: the stationary point
    # comes back exactly (also with a cross term)
    for x0, y0, hxy in [(0.2, -0.35, 0.0), (-0.45, 0.1, 0.3), (0.0, 0.0, -0.5), (0.5, -0.5, 0.2)]:
        ox, oy = O.quadratic_peak_offset(_quad_patch(x0, y0, -2.0, hxy, -1.5))
        assert ox == pytest.approx(x0, abs=1e-12) and oy == pytest.approx(y0, abs=1e-12)


def test_quadratic_offset_clamps_and_falls_back():
    # stationary point 0.8 cells away: accepted (within one cell) and clamped
    ox, oy = O.quadratic_peak_offset(_quad_patch(0.8, -0.2, -2.0, 0.0, -2.0))
    assert ox == 0.5 and oy == pytest.approx(-0.2, abs=1e-12)
    # a saddle (no maximum): 3-point parabola along x, none along y
    F = _quad_patch(0.2, 0.0, -2.0, 0.0, 2.0)
    ox, oy = O.quadratic_peak_offset(F)
    assert ox == pytest.approx(0.2, abs=1e-12) and oy == 0.0


@pytest.mark.parametrize("rho,nu", [(10.37, -5.61), (3.58, 7.44), (20.03, 0.96)])
def test_refine_recovers_noiseless_off_grid_target(rho, nu):
    # a single target whose taps all lie inside N_cp: the refined peak lands on
    # the generator's (rho, nu) within a small fraction of a fine cell
    spec = S.FrameSpec(n_sub=128, n_sym=64, qam=16, zc_root=3, n_targets=1, noise=False, on_grid=False)
    f = S.make_frame(spec, 90, 0)
    f.rho[:] = rho
    f.nu[:] = nu
    k = np.arange(128)
    l = np.arange(64)
    echo = f.b[0] * np.outer(np.exp(2j * np.pi * l * nu / 64), np.exp(-2j * np.pi * k * rho / 128))
    Y = f.A * S.tx_precoding_sequence(128, 3)[None, :] * echo
    n_pad, m_pad = 512, 256
    Hw = O.windowed_estimate(Y, f.A, n_cp=128, zc_root=3)
    P = O.frame_periodogram(Y, f.A, n_pad=n_pad, m_pad=m_pad, n_cp=128, zc_root=3)
    row, r, _ = O.find_peaks(P, 1)[0]
    s = row - m_pad // 2
    s_off, r_off = O.refine_peak(Hw, s, r, n_pad, m_pad)
    assert abs((s + s_off) * 64 / m_pad - nu) < 2e-3
    assert abs((r + r_off) * 128 / n_pad - rho) < 2e-3
    # the grid peak alone is off by up to half a padded cell
    assert abs(s * 64 / m_pad - nu) + abs(r * 128 / n_pad - rho) > 1e-2


def test_refine_peak_on_exact_fine_cell_gives_zero_offset():
    # target exactly on a padded cell: the symmetric lobe puts the fit at 0
    spec = S.FrameSpec(n_sub=64, n_sym=32, qam=4, zc_root=None, n_targets=1, noise=False)
    f = S.make_frame(spec, 91, 0)
    Hw = O.windowed_estimate(f.Y, f.A, n_cp=64)
    s, r = int(f.nu[0] * 4), int(f.rho[0] * 4)
    s_off, r_off = O.refine_peak(Hw, s, r, 256, 128)
    assert abs(s_off) < 1e-9 and abs(r_off) < 1e-9


# ------------------------------------------------------- FPS-SFT (Sec. III-C)
def _dft2_brute(h):
    n, m = h.shape
    X = np.zeros((n, m), dtype=np.complex128)
    for k1 in range(n):
        for k2 in range(m):
            acc = 0j
            for a in range(n):
                for b in range(m):
                    acc += h[a, b] * np.exp(-2j * np.pi * (k1 * a / n + k2 * b / m))
            X[k1, k2] = acc
    return X


@pytest.mark.parametrize("n,m", [(8, 4), (4, 8), (8, 8), (6, 4)])
def test_sft_slices_are_projections_of_the_2d_spectrum(n, m):
    # discrete projection-slice identity, checked term by term against a
    # brute-force 2-D DFT (also for a non-power-of-two N, Q = lcm = 12)
    rng = np.random.default_rng(30 + n + m)
    H = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    X = _dft2_brute(H.T)           # X[k1, k2], h[k, l] = H[l, k]
    dirs = O.SFT_DIRECTIONS
    S = O.sft_slices(H, dirs)
    q = O.sft_length(n, m)
    assert S.shape == (len(dirs), 3, q)
    for i, (a, b) in enumerate(dirs):
        for j, (t1, t2) in enumerate(O.SFT_OFFSETS):
            want = np.zeros(q, dtype=np.complex128)
            for k1 in range(n):
                for k2 in range(m):
                    mb = (a * k1 * (q // n) + b * k2 * (q // m)) % q
                    want[mb] += X[k1, k2] * np.exp(2j * np.pi * (k1 * t1 / n + k2 * t2 / m)) * q / (n * m)
            np.testing.assert_allclose(S[i, j], want, atol=1e-9)


@pytest.mark.parametrize("n,m,nt,seed", [(256, 64, 3, 0), (1024, 1024, 8, 0), (64, 256, 5, 1), (16, 16, 2, 0),
                                         (4096, 32, 6, 2), (32, 4096, 6, 0), (128, 128, 12, 0)])
def test_sft_recovers_noiseless_sparse_frames(n, m, nt, seed):
    spec = S.FrameSpec(n_sub=n, n_sym=m, qam=16, zc_root=3, n_targets=nt, noise=False, on_grid=True, rho_min=0,
                       rho_max=max(1, n // 4), nu_abs_max=m // 2 - 1, min_sep=1.0)
    f = S.make_frame(spec, 95, n * 10 + seed)
    det = O.fps_sft(f.Y, f.A, zc_root=3, k=nt)
    assert sorted((s, r) for s, r, _ in det) == sorted((int(v), int(r)) for r, v in zip(f.rho, f.nu))
    # the coefficient is X[k1, k2] = N M b: p = N M |b|^2
    want_p = sorted(n * m * np.abs(f.b) ** 2)
    np.testing.assert_allclose(sorted(p for _, _, p in det), want_p, rtol=1e-9)


def test_sft_peeling_resolves_collisions():
    # T1 and T2 share k1 (collide along (1, 0)); T1 and T3 share k2 (collide
    # along (0, 1) until T3, found along (1, 0), is peeled off).  Equal
    # coefficients and k2 (or k1) four apart make each collided bin fail the
    # 1-sparse test (ratio magnitude cos(pi/4)), so T1 is only found after the peel.
    n = m = 16
    comps = [(5, 3, 1.0), (5, 7, 1.0), (9, 3, 1.0)]
    k = np.arange(n)[:, None]
    l = np.arange(m)[None, :]
    h = sum(c / (n * m) * np.exp(2j * np.pi * (k1 * k / n + k2 * l / m)) for k1, k2, c in comps)
    S_ = O.sft_slices(h.T, ((1, 0), (0, 1)))
    found = O.sft_decode(S_, n, m, ((1, 0), (0, 1)), k=3)
    assert sorted((a, b) for a, b, _ in found) == [(5, 3), (5, 7), (9, 3)]
    for k1, k2, c in found:
        assert abs(c - dict(((a, b), cc) for a, b, cc in comps)[(k1, k2)]) < 1e-12


def test_sft_k_cap_takes_strongest_bin_first():
    n = m = 16
    comps = [(2, 1, 1.0), (6, 9, 3.0)]
    k = np.arange(n)[:, None]
    l = np.arange(m)[None, :]
    h = sum(c / (n * m) * np.exp(2j * np.pi * (k1 * k / n + k2 * l / m)) for k1, k2, c in comps)
    found = O.sft_decode(O.sft_slices(h.T), n, m, k=1)
    assert [(a, b) for a, b, _ in found] == [(6, 9)]


def test_sft_detection_maps_onto_the_periodogram_cell():
    # axis mapping and scale: a lone on-grid target's detection (s, r, p) is the
    # native-resolution rectangular-window periodogram's peak cell and value
    spec = S.FrameSpec(n_sub=128, n_sym=32, qam=4, zc_root=5, n_targets=1, noise=False, on_grid=True,
                       rho_min=3, rho_max=40, nu_abs_max=15)
    f = S.make_frame(spec, 99, 0)
    (s, r, p), = O.fps_sft(f.Y, f.A, zc_root=5, k=1)
    P = O.frame_periodogram(f.Y, f.A, n_pad=128, m_pad=32, n_cp=128, window_kind=O.WINDOW_RECT, zc_root=5)
    assert (s, r) == (int(f.nu[0]), int(f.rho[0]))
    assert p == pytest.approx(P[s + 16, r], rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2, 5])
def test_sft_agrees_with_periodogram_at_high_snr(seed):
    # five on-grid targets at 20 dB: FPS-SFT's cells are the periodogram's
    # top-5 local maxima (Sec. III-C compares the two on such a scene)
    spec = S.FrameSpec(n_sub=256, n_sym=64, qam=16, zc_root=1, n_targets=5, snr_db=20.0, on_grid=True,
                       rho_min=1, rho_max=60, nu_abs_max=31, min_sep=2.0)
    f = S.make_frame(spec, 96, seed)
    det = O.fps_sft(f.Y, f.A, zc_root=1, k=5)
    P = O.frame_periodogram(f.Y, f.A, n_pad=256, m_pad=64, n_cp=256, window_kind=O.WINDOW_RECT, zc_root=1)
    assert sorted((s, r) for s, r, _ in det) == sorted((row - 32, c) for row, c, _ in O.find_peaks(P, 5))


# ------------------------------------------- threshold detection (Eq. 18)
@pytest.mark.parametrize("wk,closed", [(O.WINDOW_RECT, 1.0), (O.WINDOW_HANN, 3.0 / 8.0),
                                       (O.WINDOW_HAMMING, 0.54 ** 2 + 0.46 ** 2 / 2.0)])
def test_window_energy_closed_forms(wk, closed):
    # sum of w^2 for the periodic windows: N (a0^2 + a1^2 / 2)
    for n in (16, 64, 1024):
        assert float(np.sum(O.window(n, wk) ** 2)) == pytest.approx(closed * n, rel=1e-12)


@pytest.mark.parametrize("n_cp,wk,qam", [(64, O.WINDOW_HANN, 16), (256, O.WINDOW_RECT, 4), (64, O.WINDOW_HAMMING, 16)])
def test_threshold_false_alarm_rate_on_noise(n_cp, wk, qam):
    # noise only: inside the CP range box a cell exceeds eta with probability
    # P_fa (exponential cell power); outside the box DFT-CE removed the noise
    n, m, pfa, sigma2 = 256, 64, 1e-2, 0.5
    spec = S.FrameSpec(n_sub=n, n_sym=m, qam=qam, zc_root=3, n_targets=0, snr_db=-10 * np.log10(sigma2))
    hits = tot = 0
    for i in range(6):
        f = S.make_frame(spec, 88, i)
        P = O.frame_periodogram(f.Y, f.A, n_pad=4 * n, m_pad=4 * m, n_cp=n_cp, window_kind=wk, zc_root=3)
        eta = O.cfar_threshold(f.A, sigma2, pfa, wk)
        box = P[:, 8:4 * (n_cp - 2)]  # range cells well inside [0, N_cp)
        hits += int(np.sum(box >= eta))
        tot += box.size
        # the mean cell power inside the box is sigma_P^2
        assert float(np.mean(box)) == pytest.approx(eta / -np.log(pfa), rel=0.1)
    assert hits / tot == pytest.approx(pfa, rel=0.15)


def test_threshold_detection_keeps_targets_drops_noise():
    spec = S.FrameSpec(n_sub=256, n_sym=64, qam=16, zc_root=1, n_targets=3, snr_db=-5.0, on_grid=True,
                       rho_min=1, rho_max=60, nu_abs_max=31)
    f = S.make_frame(spec, 89, 0)
    P = O.frame_periodogram(f.Y, f.A, n_pad=1024, m_pad=256, n_cp=64, zc_root=1)
    eta = O.cfar_threshold(f.A, 10 ** 0.5, 1e-6)
    det = O.detect_threshold(P, eta, 20)
    assert sorted((s - 128, r) for s, r, _ in det) == sorted((int(v * 4), int(r * 4)) for r, v in zip(f.rho, f.nu))
    assert all(v >= eta for _, _, v in det)
