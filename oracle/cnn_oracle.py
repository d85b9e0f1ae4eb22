"""FP64 CPU oracle of the CNN sub-cell peak refiner.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module; the product path
never imports, calls or links it, and it imports nothing from the product path.

The paper names machine learning as a direction for future work (Sec. V) and
gives no network.  The network written here is this build's reading of that
direction: a small convolutional regressor from a log-periodogram patch
around a detected peak to the peak's sub-cell offset.

  input   x[b, y, x, 0]: 32 x 32 patch, rows = Doppler cells, columns = range
          cells, centred on the detected cell (patch_input)
  conv1   3x3, 1 -> 32 channels, stride 1, zero padding 1, ReLU   -> 32 x 32 x 32
  conv2   3x3, 32 -> 32, stride 2, padding 1, ReLU               -> 16 x 16 x 32
  conv3   3x3, 32 -> 32, stride 1, padding 1, ReLU               -> 16 x 16 x 32
  conv4   3x3, 32 -> 32, stride 2, padding 1, ReLU               ->  8 x  8 x 32
  flatten (y * 8 + x) * 32 + c                                   -> 2048
  fc1     2048 -> 10, ReLU
  fc2     10 -> 2: (range offset, Doppler offset) in cells of the N' x M' grid

Parameters (48 576): conv weights W[co][ky][kx][ci] with bias b[co]; fc1
W[10][2048], b[10]; fc2 W[2][10], b[2].  Training minimises the mean squared
error with Adam.  Activations are NHWC: a[b, y, x, c].
"""

from __future__ import annotations

import numpy as np

PATCH = 32
CONV = (  # (name, c_in, c_out, stride)
    ("conv1", 1, 32, 1),
    ("conv2", 32, 32, 2),
    ("conv3", 32, 32, 1),
    ("conv4", 32, 32, 2),
)
FC = (("fc1", 2048, 10), ("fc2", 10, 2))


def param_shapes():
    """Ordered (name, shape) of every parameter tensor."""
    out = []
    for name, ci, co, _ in CONV:
        out += [(name + ".w", (co, 3, 3, ci)), (name + ".b", (co,))]
    for name, fi, fo in FC:
        out += [(name + ".w", (fo, fi)), (name + ".b", (fo,))]
    return out


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in param_shapes()))


def unflatten(theta: np.ndarray) -> dict:
    """Split a flat parameter vector (the order of param_shapes) into tensors."""
    theta = np.asarray(theta, dtype=np.float64)
    out, off = {}, 0
    for name, shape in param_shapes():
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].reshape(shape)
        off += n
    return out


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in param_shapes()])


# ----------------------------------------------------------------- layers
def conv_forward(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """z[b, y, x, o] = sum_{ky, kx, c} w[o, ky, kx, c] xp[b, s y + ky, s x + kx, c] + bias[o],
    xp = x zero-padded by one cell on each side."""
    n, h, wd, _ = x.shape
    ho, wo = h // stride, wd // stride
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    z = np.zeros((n, ho, wo, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            tap = xp[:, ky:ky + stride * ho:stride, kx:kx + stride * wo:stride, :]
            z += np.einsum("byxc,oc->byxo", tap, w[:, ky, kx, :])
    return z + b


def conv_backward(x: np.ndarray, w: np.ndarray, dz: np.ndarray, stride: int):
    """Gradients of conv_forward: (dx, dw, db) from dz = dL/dz."""
    n, h, wd, ci = x.shape
    ho, wo = dz.shape[1], dz.shape[2]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky, ky + stride * ho, stride), slice(kx, kx + stride * wo, stride))
            dw[:, ky, kx, :] = np.einsum("byxo,byxc->oc", dz, xp[sl])
            dxp[sl] += np.einsum("byxo,oc->byxc", dz, w[:, ky, kx, :])
    return dxp[:, 1:-1, 1:-1, :], dw, dz.sum(axis=(0, 1, 2))


def relu(z):
    return np.maximum(z, 0.0)


def forward(params: dict, x: np.ndarray):
    """x: [B, 32, 32] (or [B, 32, 32, 1]).  Returns (output [B, 2], cache)."""
    a = np.asarray(x, dtype=np.float64)
    if a.ndim == 3:
        a = a[..., None]
    cache = {"in": a}
    for name, _, _, stride in CONV:
        z = conv_forward(a, params[name + ".w"], params[name + ".b"], stride)
        a = relu(z)
        cache[name] = (z, a)
    f = a.reshape(a.shape[0], -1)
    cache["flat"] = f
    z1 = f @ params["fc1.w"].T + params["fc1.b"]
    a1 = relu(z1)
    cache["fc1"] = (z1, a1)
    out = a1 @ params["fc2.w"].T + params["fc2.b"]
    return out, cache


def backward(params: dict, cache: dict, dout: np.ndarray) -> dict:
    """Gradients of every parameter from dL/d(output), by the chain rule
    through forward in reverse."""
    g = {}
    z1, a1 = cache["fc1"]
    g["fc2.w"] = dout.T @ a1
    g["fc2.b"] = dout.sum(axis=0)
    da1 = dout @ params["fc2.w"]
    dz1 = da1 * (z1 > 0)
    g["fc1.w"] = dz1.T @ cache["flat"]
    g["fc1.b"] = dz1.sum(axis=0)
    df = dz1 @ params["fc1.w"]
    da = df.reshape(cache["conv4"][1].shape)
    for i in range(len(CONV) - 1, -1, -1):
        name, _, _, stride = CONV[i]
        z, _ = cache[name]
        dz = da * (z > 0)
        x_in = cache[CONV[i - 1][0]][1] if i > 0 else cache["in"]
        da, g[name + ".w"], g[name + ".b"] = conv_backward(x_in, params[name + ".w"], dz, stride)
    return g


def mse(pred: np.ndarray, label: np.ndarray):
    """L = mean over the batch and both outputs of (pred - label)^2, and dL/dpred."""
    d = np.asarray(pred, dtype=np.float64) - np.asarray(label, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_step(theta, grad, m, v, t: int, lr: float):
    """One Adam update (Kingma and Ba) of flat vectors; t counts from 1.
    Returns (theta, m, v)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * grad
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * grad * grad
    mhat = m / (1.0 - ADAM_B1 ** t)
    vhat = v / (1.0 - ADAM_B2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + ADAM_EPS), m, v


# ------------------------------------------------------------ patches
def patch_input(P: np.ndarray, row: int, r: int) -> np.ndarray:
    """The 32 x 32 log-periodogram patch around cell (row, r) of P ([M'][N'],
    cyclic in both axes): rows row-16 .. row+15, columns r-16 .. r+15,
    ln(max(P, 1e-12 P_c)) - ln P_c with P_c = P[row, r] (the floor keeps the
    exact zeros of DFT-CE finite)."""
    mp, nq = P.shape
    rows = (row + np.arange(-PATCH // 2, PATCH // 2)) % mp
    cols = (r + np.arange(-PATCH // 2, PATCH // 2)) % nq
    w = np.asarray(P, dtype=np.float64)[np.ix_(rows, cols)]
    pc = float(P[row, r])
    return np.log(np.maximum(w, 1e-12 * pc)) - np.log(pc)
