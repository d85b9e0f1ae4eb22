"""Pins of the FP64 CNN oracle: brute-force convolution, finite-difference
gradients of the whole network, Adam's closed form on its first step, and
the patch definition."""

import numpy as np
import pytest

from oracle import cnn_oracle as C
from oracle import radar_oracle as O
from synth import cnn_init
from synth import frames as S


def test_parameter_count_and_layout():
    assert C.n_params() == 48576 == cnn_init.N_PARAMS
    shapes = [int(np.prod(s)) for _, s in C.param_shapes()]
    assert shapes == [c for _, c in cnn_init.LAYOUT]
    th = cnn_init.init_params(0)
    np.testing.assert_array_equal(C.flatten(C.unflatten(th)), th.astype(np.float64))


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_forward_brute_force(stride):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 6, 4, 3))
    w = rng.standard_normal((5, 3, 3, 3))
    b = rng.standard_normal(5)
    z = C.conv_forward(x, w, b, stride)
    assert z.shape == (2, 6 // stride, 4 // stride, 5)
    for n in range(2):
        for y in range(6 // stride):
            for xx in range(4 // stride):
                for o in range(5):
                    acc = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            iy, ix = stride * y + ky - 1, stride * xx + kx - 1
                            if 0 <= iy < 6 and 0 <= ix < 4:
                                acc += sum(w[o, ky, kx, c] * x[n, iy, ix, c] for c in range(3))
                    assert z[n, y, xx, o] == pytest.approx(acc, abs=1e-12)


def _loss(theta, x, lab):
    out, _ = C.forward(C.unflatten(theta), x)
    return C.mse(out, lab)[0]


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    theta = cnn_init.init_params(3).astype(np.float64)
    theta[[i for i in range(len(theta)) if i % 7 == 0]] += 0.01  # non-zero biases too
    x = rng.standard_normal((3, 32, 32))
    lab = rng.standard_normal((3, 2))
    params = C.unflatten(theta)
    out, cache = C.forward(params, x)
    _, dout = C.mse(out, lab)
    g = C.flatten(C.backward(params, cache, dout))
    # every tensor: a few coordinates by central differences
    off = 0
    for name, shape in C.param_shapes():
        n = int(np.prod(shape))
        for j in rng.choice(n, size=min(n, 4), replace=False):
            i = off + int(j)
            h = 1e-5
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            fd = (_loss(tp, x, lab) - _loss(tm, x, lab)) / (2 * h)
            assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, j)
        off += n


def test_mse_gradient():
    pred = np.array([[1.0, -2.0], [0.5, 3.0]])
    lab = np.array([[0.0, -1.0], [1.0, 1.0]])
    L, d = C.mse(pred, lab)
    assert L == pytest.approx((1 + 1 + 0.25 + 4) / 4)
    np.testing.assert_allclose(d, 2 * (pred - lab) / 4)


def test_adam_first_steps_closed_form():
    # first step: m_hat = g, v_hat = g^2, so the move is lr * g / (|g| + eps)
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = C.adam_step(th, g, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(t1, th - 0.01 * g / (np.abs(g) + C.ADAM_EPS), rtol=1e-12)
    # second step with the same gradient moves by the same amount
    t2, _, _ = C.adam_step(t1, g, m, v, 2, 0.01)
    np.testing.assert_allclose(t2 - t1, t1 - th, rtol=1e-9)


def test_patch_input_definition():
    f = S.make_frame(S.spec_small(snr_db=10.0), 1, 0)
    P = O.frame_periodogram(f.Y, f.A, n_pad=1024, m_pad=256, n_cp=32, zc_root=1)
    row, r, _ = O.find_peaks(P, 1)[0]
    x = C.patch_input(P, row, r)
    assert x.shape == (32, 32) and x[16, 16] == 0.0
    assert np.all(x[15:18, 15:18] <= 0.0)  # a local maximum
    # cyclic: a corner cell wraps round both axes
    x0 = C.patch_input(P, 0, 0)
    assert x0[0, 0] == pytest.approx(np.log(max(P[-16, -16], 1e-12 * P[0, 0])) - np.log(P[0, 0]))


def test_forward_composition_hand_worked():
    """The network's composition (the layer order, the stride-2 sampling, the
    NHWC flatten index (y * 8 + x) * 32 + c, ReLU after fc1 but not after fc2,
    the biases) on hand-set weights that route single pixels through single
    channels, against an output worked out by hand:

      x[8][12] = 1.5, x[20][4] = -5, x[0][0] = 100 (routed nowhere)
      conv1  ch0 = relu(x), ch1 = relu(-x)          (centre taps)
      conv2  ch0 <- ch0, ch5 <- ch1                  (stride 2: reads row 2y, col 2x)
      conv3  ch0 <- ch0, ch5 <- ch5, ch9 = bias 0.75 everywhere
      conv4  ch0 <- ch0, ch7 <- ch5 (stride 2), ch9 = relu(2 * 0.75 - 0.5) = 1
      so x[8][12] lands at conv4 (2, 3, ch0) = 1.5 and x[20][4] at (5, 1, ch7) = 5
      flat   (2*8+3)*32+0 = 608,  (5*8+1)*32+7 = 1319,  (7*8+7)*32+9 = 2025
      fc1    a0 = relu(2*1.5 + 0.5) = 3.5, a1 = relu(5 - 3) = 2, a2 = relu(-1) = 0,
             a3 = relu(-1.5) = 0, a4 = relu(1) = 1
      fc2    out0 = 3.5 + 3*2 + 10*0 + 7*0 + 0.125*1 + 0.25 = 9.875
             out1 = -3.5 + 0.5*2 - 2 = -4.5  (no ReLU: stays negative)"""
    p = {name: np.zeros(shape) for name, shape in C.param_shapes()}
    p["conv1.w"][0, 1, 1, 0] = 1.0
    p["conv1.w"][1, 1, 1, 0] = -1.0
    p["conv2.w"][0, 1, 1, 0] = 1.0
    p["conv2.w"][5, 1, 1, 1] = 1.0
    p["conv3.w"][0, 1, 1, 0] = 1.0
    p["conv3.w"][5, 1, 1, 5] = 1.0
    p["conv3.b"][9] = 0.75
    p["conv4.w"][0, 1, 1, 0] = 1.0
    p["conv4.w"][7, 1, 1, 5] = 1.0
    p["conv4.w"][9, 1, 1, 9] = 2.0
    p["conv4.b"][9] = -0.5
    p["fc1.w"][0, 608], p["fc1.b"][0] = 2.0, 0.5
    p["fc1.w"][1, 1319], p["fc1.b"][1] = 1.0, -3.0
    p["fc1.b"][2] = -1.0
    p["fc1.w"][3, 608] = -1.0
    p["fc1.w"][4, 2025] = 1.0
    p["fc2.w"][0, :5] = [1.0, 3.0, 10.0, 7.0, 0.125]
    p["fc2.b"][0] = 0.25
    p["fc2.w"][1, :2] = [-1.0, 0.5]
    p["fc2.b"][1] = -2.0
    x = np.zeros((1, 32, 32))
    x[0, 8, 12], x[0, 20, 4], x[0, 0, 0] = 1.5, -5.0, 100.0
    out, cache = C.forward(p, x)
    np.testing.assert_allclose(cache["fc1"][1][0, :5], [3.5, 2.0, 0.0, 0.0, 1.0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(out[0], [9.875, -4.5], rtol=0, atol=1e-12)
