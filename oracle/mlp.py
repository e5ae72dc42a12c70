"""Float64 Fourier-feature MLP with a hand-written backward pass.

Test infrastructure: see the package docstring.

The paper motivates machine learning for faster propagation prediction
(Sec. I, and the remarks closing Sec. III-A) but specifies no network.  The
surrogate here is fixed as follows (the GPU kernels implement the same
function in bf16/fp32):

* input v in R^5: transmitter (x, y, z) and cell centre (x, y), each mapped
  affinely to about [-1, 1] by (p - centre) / half_extent;
* Fourier features gamma(v) = [sin(2 pi B v), cos(2 pi B v)], B in R^{64x5};
* 4 hidden layers of width 256, h_l = gelu(W_l h_{l-1} + b_l), with the tanh
  form gelu(x) = x / 2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)));
* linear head y = w_5 . h_4 + b_5, plus optionally the free-space gain of the
  link, 20 log10(c0 / (4 pi f d)) (Friis with isotropic antennas, Sec. II-A),
  so that the network learns the residual (path gain in dB);
* loss = sum_i m_i (y_i - t_i)^2 / sum_i m_i (mask m_i in {0, 1}).

Parameter vector layout (float32 on the GPU, float64 here):
W1[256][128], b1[256], W2[256][256], b2, W3, b3, W4, b4, w5[256], b5[1].
"""
from __future__ import annotations

import numpy as np

from .consts import C0

N_IN = 5
N_FREQ = 64
HIDDEN = 256
LAYERS = 4
C_GELU = np.sqrt(2.0 / np.pi)


def layer_shapes():
    shapes = []
    fan_in = 2 * N_FREQ
    for _ in range(LAYERS):
        shapes.append(((HIDDEN, fan_in), (HIDDEN,)))
        fan_in = HIDDEN
    shapes.append(((1, HIDDEN), (1,)))
    return shapes


def param_count():
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in layer_shapes())


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for w, b in layer_shapes():
        nw, nb = int(np.prod(w)), int(np.prod(b))
        out.append((theta[k:k + nw].reshape(w), theta[k + nw:k + nw + nb]))
        k += nw + nb
    assert k == theta.size
    return out


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(C_GELU * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    u = C_GELU * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    du = C_GELU * (1.0 + 3 * 0.044715 * x ** 2)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du


# Map inference (reading R21 of the design notes): GELU is evaluated there as
# x clamp(1/2 + u Q(u^2), 0, 1) with u = clamp(x / 4, -1, 1) and Q the degree-6
# least-squares fit below (coefficients of u^0 .. u^12 in powers of u^2).
GELU_POLY = (1.59098072, -4.1370718, 9.05178404, -13.5802262, 12.9487521, -6.98037448, 1.60618985)


def gelu_poly(x):
    u = np.clip(np.asarray(x, dtype=np.float64) / 4.0, -1.0, 1.0)
    return x * np.clip(0.5 + u * np.polyval(GELU_POLY[::-1], u * u), 0.0, 1.0)


def round_weights_f16(theta):
    """theta with W1..W4 and w5 rounded to IEEE half precision (round to
    nearest), the weight format of map inference: layer 1 is stored as W1 / 4
    and the head as 4 w5 (powers of two, so only the subnormal range differs
    from rounding W itself); biases stay as they are."""
    layers = unpack(theta)
    out = []
    for li, (W, b) in enumerate(layers):
        sc = 0.25 if li == 0 else (4.0 if li == len(layers) - 1 else 1.0)
        out.append((np.asarray(np.float16(sc * W), dtype=np.float64) / sc, b))
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in out])


def features(v, Bf):
    proj = 2.0 * np.pi * (np.asarray(v, dtype=np.float64) @ np.asarray(Bf, dtype=np.float64).T)
    return np.concatenate([np.sin(proj), np.cos(proj)], axis=1)


def free_space_db(points, freq_hz, rx_z):
    """Free-space gain [dB] from the transmitter (points[:, 0:3]) to the cell
    centre (points[:, 3], points[:, 4], rx_z): 20 log10(lambda / (4 pi d))."""
    p = np.asarray(points, dtype=np.float64)
    d = np.sqrt((p[:, 3] - p[:, 0]) ** 2 + (p[:, 4] - p[:, 1]) ** 2 + (rx_z - p[:, 2]) ** 2)
    return 20.0 * np.log10(C0 / freq_hz / (4.0 * np.pi * d))


def forward(theta, v, Bf, feats=None, prior_db=None, act=gelu):
    """Prediction and the cache for ``backward``; prior_db (per row, e.g. from
    ``free_space_db``) is added to the head's output; act is the activation
    (``gelu``, or ``gelu_poly`` for the map-inference reading; ``backward``
    assumes ``gelu``)."""
    layers = unpack(theta)
    h = features(v, Bf) if feats is None else np.asarray(feats, dtype=np.float64)
    cache = [h]
    for W, b in layers[:-1]:
        z = h @ W.T + b
        h = act(z)
        cache.append((z, h))
    w5, b5 = layers[-1]
    y = h @ w5[0] + b5[0]
    if prior_db is not None:
        y = y + np.asarray(prior_db, dtype=np.float64)
    return y, cache


def loss(y, t, m):
    m = np.asarray(m, dtype=np.float64)
    return float(np.sum(m * (y - t) ** 2) / np.sum(m))


def backward(theta, cache, y, t, m):
    """d loss / d theta (float64, same layout as theta)."""
    layers = unpack(theta)
    m = np.asarray(m, dtype=np.float64)
    g = 2.0 * m * (y - t) / np.sum(m)                   # d loss / d y
    grads = []
    h4 = cache[-1][1]
    w5 = layers[-1][0]
    grads.append((g @ h4, np.array([g.sum()])))          # w5, b5
    dh = np.outer(g, w5[0])
    for li in range(LAYERS - 1, -1, -1):
        z, _ = cache[li + 1]
        h_prev = cache[li] if li == 0 else cache[li][1]
        dz = dh * gelu_grad(z)
        W = layers[li][0]
        grads.append((dz.T @ h_prev, dz.sum(axis=0)))
        dh = dz @ W
    grads = grads[::-1]
    flat = []
    for (gw, gb) in grads:
        flat.append(np.asarray(gw).reshape(-1))
        flat.append(np.asarray(gb).reshape(-1))
    return np.concatenate(flat)


def normalize(points, centre, half):
    return (np.asarray(points, dtype=np.float64) - np.asarray(centre)) / np.asarray(half)
