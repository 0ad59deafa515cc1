"""Float64 reference of the spectral-scaling network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper proposes no network; the nearest idea is its closing remark on
learning on the fly (a network that decides whether an observable can be taken
from the model or must be computed, and is retrained on the computed cases).
Here a small multilayer perceptron predicts, from 16 cheap per-submatrix
features, the logarithm of two spectral bounds relative to the Gershgorin
bound.  Its prediction is only used after a power-iteration guard accepts it.

Architecture and conventions (shared with the GPU kernels by specification,
not by code):
    x  = (features - mean) / std                       (16)
    h1 = tanh(W1 x + b1)                                (64)
    h2 = tanh(W2 h1 + b2)                               (64)
    y  = W3 h2 + b3                                     (2)
    loss = 1/n sum_samples sum_outputs (y - t)^2
Parameters are packed into one vector in the order W1 (64x16, row-major), b1,
W2 (64x64), b2, W3 (2x64), b3: 5378 values.  Adam (Kingma & Ba 2015) with
beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 16, 64, 2
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta: np.ndarray, x: np.ndarray):
    """x: (n, 16) already normalised.  Returns y (n, 2) and the activations."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(x @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    return y, (x, h1, h2)


def loss(theta, x, t) -> float:
    y, _ = forward(theta, x)
    return float(np.sum((y - t) ** 2) / x.shape[0])


def grad(theta, x, t):
    """Loss and its gradient by the chain rule (backpropagation)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    y, (x, h1, h2) = forward(theta, x)
    n = x.shape[0]
    dy = 2.0 * (y - t) / n                   # (n, 2)
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(0)
    dh2 = dy @ p["W3"]                       # (n, 64)
    dz2 = dh2 * (1.0 - h2 * h2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return float(np.sum((y - t) ** 2) / n), pack(g)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t = 1-based step count).  Returns new theta, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, numpy
    default_rng(seed), drawn in packing order."""
    rng = np.random.default_rng(seed)
    parts = []
    fan = {"W1": N_IN, "b1": N_IN, "W2": N_H, "b2": N_H, "W3": N_H, "b3": N_H}
    for name, shp in SHAPES:
        a = 1.0 / np.sqrt(fan[name])
        parts.append(rng.uniform(-a, a, size=shp).ravel())
    return np.concatenate(parts)
