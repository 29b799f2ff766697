"""FP64 reference for the learned cost model's network.

TEST INFRASTRUCTURE ONLY.  A plain numpy forward / backward / Adam step of
the 16 -> 64 -> 64 -> 2 perceptron whose GPU kernels schedule queries
(the network predicts log1p(node visits) and log1p(neighbour count) of a
query block; it never decides an edge).

Layout (row-major, the same as the GPU kernels' parameter buffer):
  W1 [64,16], b1 [64], W2 [64,64], b2 [64], W3 [2,64], b3 [2]
Activation: SiLU, silu(z) = z * sigmoid(z).  Loss: mean over the batch of
the sum over the two outputs of the squared error, halved:
  L = (1 / (2B)) * sum_b sum_o (y_bo - t_bo)^2.
"""
from __future__ import annotations

import numpy as np

SIZES = (16, 64, 64, 2)
SHAPES = (("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
          ("W3", (2, 64)), ("b3", (2,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 5378


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).ravel()
                           for name, _ in SHAPES])


def init(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            p[name] = rng.normal(0.0, np.sqrt(1.0 / shp[1]), shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p)


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(theta: np.ndarray, x: np.ndarray):
    p = unpack(np.asarray(theta, np.float64))
    x = np.asarray(x, np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = z1 * _sig(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = z2 * _sig(z2)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(theta, x, t) -> float:
    y, _ = forward(theta, x)
    B = y.shape[0]
    return float(0.5 * np.sum((y - np.asarray(t, np.float64)) ** 2) / B)


def _dsilu(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def backward(theta, x, t):
    """Gradient of ``loss`` with respect to the packed parameters."""
    p = unpack(np.asarray(theta, np.float64))
    y, (x, z1, h1, z2, h2) = forward(theta, x)
    B = y.shape[0]
    gy = (y - np.asarray(t, np.float64)) / B
    g = {"W3": gy.T @ h2, "b3": gy.sum(0)}
    gh2 = gy @ p["W3"]
    gz2 = gh2 * _dsilu(z2)
    g["W2"] = gz2.T @ h1
    g["b2"] = gz2.sum(0)
    gh1 = gz2 @ p["W2"]
    gz1 = gh1 * _dsilu(z1)
    g["W1"] = gz1.T @ x
    g["b1"] = gz1.sum(0)
    return pack(g)


def adam_step(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, bias-corrected); returns new
    (theta, m, v).  ``step`` counts from 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def finite_diff(theta, x, t, idx, h=1e-6):
    """Central difference of the loss in the listed parameter coordinates."""
    out = np.empty(len(idx))
    for k, i in enumerate(idx):
        tp = np.array(theta, np.float64)
        tm = np.array(theta, np.float64)
        tp[i] += h
        tm[i] -= h
        out[k] = (loss(tp, x, t) - loss(tm, x, t)) / (2 * h)
    return out
