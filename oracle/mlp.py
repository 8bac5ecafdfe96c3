"""FP64 oracle of the learned-step perceptron -- TEST INFRASTRUCTURE ONLY.

A 5-64-64-1 perceptron with ReLU hidden layers, y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3,
its mean-squared training loss L = 1/(2n) sum_i (y_i - t_i)^2, the gradient of L by the
chain rule (the ReLU derivative is taken as 1 where the pre-activation is > 0, else 0),
and one Adam update (Kingma and Ba, 2015: biased first and second moment estimates,
bias-corrected by 1 - beta^step).  The parameter vector is ordered W1[64][5], b1[64],
W2[64][64], b2[64], w3[64], b3, row-major.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 5, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("w3", (N_H,)), ("b3", ())]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    """Split the flat parameter vector into named FP64 arrays."""
    p = np.asarray(p, dtype=np.float64).ravel()
    assert p.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape) if shape else p[o]
        o += k
    return out


def pack(d) -> np.ndarray:
    return np.concatenate([np.atleast_1d(np.asarray(d[name], dtype=np.float64)).ravel() for name, _ in SIZES])


def forward(p, X):
    """Outputs y [n] and the intermediate pre-activations (FP64)."""
    q = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ q["W1"].T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ q["w3"] + q["b3"]
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(p, X, t):
    """(L, dL/dp) with L = 1/(2n) sum (y - t)^2, by the chain rule layer by layer."""
    q = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    n = X.shape[0]
    e = y - np.asarray(t, dtype=np.float64)
    L = 0.5 * float(e @ e) / n
    dy = e / n                                  # dL/dy
    g = {"w3": h2.T @ dy, "b3": dy.sum()}
    dz2 = np.outer(dy, q["w3"]) * (z2 > 0)      # dL/dz2
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ q["W2"]) * (z1 > 0)            # dL/dz1
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g)


def adam_step(p, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update; returns (p, m, v) as new FP64 arrays."""
    p, grad = np.asarray(p, dtype=np.float64), np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * grad
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
