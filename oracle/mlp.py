"""Numpy FP64 reference of the block-rank MLP (test infrastructure only).

The paper shows the local rank of every block of its H-matrix but does not predict ranks; this
is the reference for the learned part built around the compression: a 4 -> 64 -> 64 -> 1
multilayer perceptron with ReLU activations that maps standardized block features to
ln(1 + rank), trained with the mean squared error and Adam.

Parameter vector layout (4545 entries), shared with the device code's interface:
  W1 (64 x 4, row-major) | b1 (64) | W2 (64 x 64, row-major) | b2 (64) | W3 (64) | b3 (1)
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 4, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 4545


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in SIZES])


def he_init(seed: int):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.standard_normal((N_H, N_IN)) * np.sqrt(2.0 / N_IN), "b1": np.zeros(N_H),
         "W2": rng.standard_normal((N_H, N_H)) * np.sqrt(2.0 / N_H), "b2": np.zeros(N_H),
         "W3": rng.standard_normal(N_H) * np.sqrt(2.0 / N_H), "b3": np.zeros(1)}
    return pack(p)


def forward(theta, X):
    """Returns the prediction (n) and the cached activations."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ p["W3"] + p["b3"][0]
    return o, (X, z1, h1, z2, h2)


def loss_and_grad(theta, X, y):
    """Mean squared error (1/n) sum (o - y)^2 and its gradient with respect to theta."""
    p = unpack(theta)
    o, (X, z1, h1, z2, h2) = forward(theta, X)
    n = X.shape[0]
    r = o - y
    loss = float((r * r).sum() / n)
    do = 2.0 * r / n
    g = {"W3": h2.T @ do, "b3": np.array([do.sum()])}
    dz2 = np.outer(do, p["W3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) at step t >= 1; returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def block_features(m, n, diam_t, diam_s, dist, k):
    """Raw features of far blocks: log2 m, log2 n, ln(dist / max diam), k max diam / (2 pi)."""
    m = np.asarray(m, np.float64)
    n = np.asarray(n, np.float64)
    dmax = np.maximum(np.maximum(diam_t, diam_s), 1e-12)
    return np.stack([np.log2(m), np.log2(n), np.log(np.maximum(dist, 1e-12) / dmax),
                     k * dmax / (2 * np.pi)], 1)
