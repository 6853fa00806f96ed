"""FP64 reference of the learned preconditioner's network and its training step.
Test infrastructure only; the HIP library has its own kernels.

Network: 12 -> 64 -> 64 -> 1 with tanh hidden layers,
  h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = w3 . h2 + b3.
Loss over a batch: mean of (y - target)^2.  Optimiser: Adam (Kingma & Ba 2015)
with bias correction.  Parameter layout (5,057 values): W1 [64][12], b1 [64],
W2 [64][64], b2 [64], w3 [64], b3 [1].
"""
from __future__ import annotations

import numpy as np

D_IN, D_H = 12, 64
SIZES = (("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)), ("w3", (D_H,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = flat[o:o + k].reshape(shape)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init(seed=0):
    """Glorot-uniform weights, zero biases (the initial parameters are an input
    to both implementations)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SIZES:
        if name.startswith("b"):
            p[name] = np.zeros(shape)
        else:
            fan_in = shape[-1] if len(shape) == 2 else D_H
            fan_out = shape[0] if len(shape) == 2 else 1
            lim = np.sqrt(6.0 / (fan_in + fan_out))
            p[name] = rng.uniform(-lim, lim, size=shape)
    return pack(p)


def forward(flat, X):
    p = unpack(flat)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (X, h1, h2)


def loss_and_grad(flat, X, target):
    """MSE loss and its gradient by back-propagation through the two tanh layers."""
    p = unpack(flat)
    y, (X, h1, h2) = forward(flat, X)
    B = X.shape[0]
    r = y - np.asarray(target, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    d2 = np.outer(dy, p["w3"]) * (1.0 - h2 * h2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 * h1)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(axis=0)
    return loss, pack(g)


def adam_step(flat, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1).  Returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
