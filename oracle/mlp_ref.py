"""FP64 reference of the learned cost model: TEST INFRASTRUCTURE ONLY.

The cost model is not in the paper: the paper's Section 8 learns one variant
per processor and names a run-time, per-query optimizer as future work
(Sections 9.3.4 and 9.4). The model here predicts ln(run time in ms) of a (query,
variant) pair from 12 features:

    z1 = W1 @ ((x - mu) / sd) + b1,  h1 = relu(z1)        (64 units)
    z2 = W2 @ h1 + b2,               h2 = relu(z2)        (64 units)
    yhat = W3 @ h2 + b3                                   (1 output)

Loss: mean squared error over a batch, L = mean((yhat - y)^2). Optimiser:
Adam (Kingma & Ba 2015) with bias correction.

Flat parameter layout (5,057 values): W1 (64x12, row-major), b1 (64),
W2 (64x64, row-major), b2 (64), W3 (64), b3 (1).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 12, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[n], dtype=np.float64).ravel() for n, _ in SIZES])


def forward(theta, X, mu, sd):
    """Predictions and the intermediate values backprop needs."""
    p = unpack(theta)
    xn = (np.asarray(X, dtype=np.float64) - mu) / sd
    z1 = xn @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    yhat = h2 @ p["W3"] + p["b3"][0]
    return yhat, (xn, z1, h1, z2, h2)


def loss(theta, X, y, mu, sd):
    yhat, _ = forward(theta, X, mu, sd)
    return float(np.mean((yhat - np.asarray(y, dtype=np.float64)) ** 2))


def grad(theta, X, y, mu, sd):
    """Gradient of the mean squared error, by the chain rule written out layer by layer."""
    p = unpack(theta)
    yhat, (xn, z1, h1, z2, h2) = forward(theta, X, mu, sd)
    m = len(yhat)
    d3 = 2.0 * (yhat - np.asarray(y, dtype=np.float64)) / m          # dL/dyhat
    g = {"W3": d3 @ h2, "b3": np.array([d3.sum()])}
    d2 = np.outer(d3, p["W3"]) * (z2 > 0)                             # dL/dz2
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (z1 > 0)                                    # dL/dz1
    g["W1"] = d1.T @ xn
    g["b1"] = d1.sum(axis=0)
    return pack(g), float(np.mean((yhat - y) ** 2))


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init(seed=0):
    """He-style initialisation used by the tests (the library draws its own)."""
    rng = np.random.default_rng(seed)
    parts = {"W1": rng.normal(0, np.sqrt(2 / N_IN), (N_H, N_IN)), "b1": np.zeros(N_H),
             "W2": rng.normal(0, np.sqrt(2 / N_H), (N_H, N_H)), "b2": np.zeros(N_H),
             "W3": rng.normal(0, np.sqrt(1 / N_H), N_H), "b3": np.zeros(1)}
    return pack(parts)
