"""Plain FP64 reference of the cost model's MLP -- TEST INFRASTRUCTURE ONLY.

Model: 24 standardized features -> 64 (ReLU) -> 64 (ReLU) -> 1 (linear),
predicting log runtime.  Loss: mean squared error over the batch.  Optimizer:
Adam (Kingma and Ba, ICLR 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
full batch, bias-corrected moments.

Parameter vector layout (5825 values), shared with the library:
W1 (64 x 24, row = output unit), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1).
"""
from __future__ import annotations

import numpy as np

N_IN, H = 24, 64
SIZES = [("W1", (H, N_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def standardize(X, mean=None, std=None):
    """(X - mean) / std per feature; std of a constant feature is taken as 1."""
    X = np.asarray(X, dtype=np.float64)
    if mean is None:
        mean = X.mean(axis=0)
        std = X.std(axis=0)
        std = np.where(std > 0, std, 1.0)
    return (X - mean) / std, mean, std


def forward(theta, Xs):
    p = unpack(theta)
    z1 = Xs @ p["W1"].T + p["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = np.maximum(z2, 0.0)
    y = a2 @ p["w3"] + p["b3"][0]
    return y, (z1, a1, z2, a2)


def loss(theta, Xs, t):
    y, _ = forward(theta, Xs)
    return float(np.mean((y - t) ** 2))


def grad(theta, Xs, t):
    """Gradient of the mean squared error by the chain rule."""
    p = unpack(theta)
    y, (z1, a1, z2, a2) = forward(theta, Xs)
    n = Xs.shape[0]
    dy = 2.0 * (y - t) / n
    g = {}
    g["w3"] = a2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, p["w3"]) * (z2 > 0)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ Xs
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def adam_step(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta0, X, t, epochs, lr):
    """Standardize X, then `epochs` full-batch Adam steps.  Returns
    (theta, mean, std, loss before each step)."""
    Xs, mean, std = standardize(X)
    theta = np.asarray(theta0, dtype=np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    for e in range(1, epochs + 1):
        hist.append(loss(theta, Xs, t))
        theta, m, v = adam_step(theta, m, v, grad(theta, Xs, t), e, lr)
    return theta, mean, std, np.array(hist)


def predict(theta, mean, std, X):
    Xs, _, _ = standardize(X, mean, std)
    return forward(theta, Xs)[0]
