"""Pins of the FP64 perceptron oracle (learned initial step): central finite differences
of the loss (piecewise quadratic in each parameter, so the central difference is exact
away from ReLU kinks), closed forms of degenerate networks, and Adam's closed-form first
steps."""
import numpy as np
import pytest

import synthetic as syn
from oracle import mlp


def _data(n=40, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, mlp.N_IN))
    t = rng.standard_normal(n)
    return X, t


def test_layout_and_count():
    p = syn.mlp_params(1)
    assert p.size == mlp.N_PARAMS == 64 * 5 + 64 + 64 * 64 + 64 + 64 + 1
    q = mlp.unpack(p)
    assert q["W1"].shape == (64, 5) and q["W2"].shape == (64, 64) and q["w3"].shape == (64,)
    assert np.array_equal(mlp.pack(q), p.astype(np.float64))


def test_forward_by_loops():
    p = syn.mlp_params(2).astype(np.float64)
    q = mlp.unpack(p)
    X, _ = _data(5, seed=1)
    y, _ = mlp.forward(p, X)
    for s in range(5):
        h1 = [max(0.0, sum(q["W1"][i, k] * X[s, k] for k in range(5)) + q["b1"][i]) for i in range(64)]
        h2 = [max(0.0, sum(q["W2"][j, i] * h1[i] for i in range(64)) + q["b2"][j]) for j in range(64)]
        ys = sum(q["w3"][j] * h2[j] for j in range(64)) + q["b3"]
        assert y[s] == pytest.approx(ys, rel=1e-12, abs=1e-12)


def test_gradient_central_differences():
    p = syn.mlp_params(3).astype(np.float64)
    p += np.random.default_rng(4).uniform(-0.05, 0.05, p.size)   # nonzero biases
    X, t = _data(40, seed=5)
    L, g = mlp.loss_and_grad(p, X, t)
    rng = np.random.default_rng(6)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 300, replace=False), [mlp.N_PARAMS - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, t)[0] - mlp.loss_and_grad(p - e, X, t)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], abs=1e-7 * max(1.0, np.abs(g).max())), i
    assert L == pytest.approx(0.5 * np.mean((mlp.forward(p, X)[0] - t) ** 2), rel=1e-14)


def test_dead_network_closed_form():
    # all weights and hidden biases zero: y = b3 for every input, dL/db3 = mean(b3 - t), and
    # every other derivative vanishes (no pre-activation is > 0)
    p = np.zeros(mlp.N_PARAMS)
    p[-1] = 0.7
    X, t = _data(30, seed=7)
    L, g = mlp.loss_and_grad(p, X, t)
    assert L == pytest.approx(0.5 * np.mean((0.7 - t) ** 2), rel=1e-14)
    assert g[-1] == pytest.approx(np.mean(0.7 - t), rel=1e-14)
    assert np.all(g[:-1] == 0.0)


def test_identity_regime_is_linear_least_squares():
    # hidden biases large enough that every pre-activation is positive: the network is the
    # affine map y = w3.(W2 (W1 x + b1) + b2) + b3, so dL/dw3 = 1/n sum e h2 and dL/db3 = mean(e)
    p = syn.mlp_params(8).astype(np.float64) * 0.01
    q = mlp.unpack(p)
    q["b1"] = np.full(64, 10.0)
    q["b2"] = np.full(64, 10.0)
    p = mlp.pack(q)
    X, t = _data(25, seed=9)
    L, g = mlp.loss_and_grad(p, X, t)
    h1 = X @ q["W1"].T + q["b1"]
    h2 = h1 @ q["W2"].T + q["b2"]
    e = h2 @ q["w3"] + q["b3"] - t
    gq = mlp.unpack(g)
    assert np.allclose(gq["w3"], h2.T @ e / 25, rtol=1e-12, atol=1e-14)
    assert gq["b3"] == pytest.approx(e.mean(), rel=1e-12)
    assert np.allclose(gq["W1"], np.outer(q["W2"].T @ q["w3"], X.T @ e / 25), rtol=1e-10, atol=1e-15)


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(10)
    p = rng.standard_normal(50)
    g1 = rng.standard_normal(50)
    p1, m1, v1 = mlp.adam_step(p, g1, np.zeros(50), np.zeros(50), 1, lr=1e-2, eps=1e-8)
    # after one step the bias-corrected moments are g and g^2
    assert np.allclose(p1, p - 1e-2 * g1 / (np.abs(g1) + 1e-8), rtol=1e-14, atol=1e-16)
    g2 = rng.standard_normal(50)
    p2, m2, v2 = mlp.adam_step(p1, g2, m1, v1, 2, lr=1e-2, eps=1e-8)
    mh = (0.9 * 0.1 * g1 + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    assert np.allclose(p2, p1 - 1e-2 * mh / (np.sqrt(vh) + 1e-8), rtol=1e-13, atol=1e-16)


def test_adam_training_fits_a_smooth_target():
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, (200, 5))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    p = syn.mlp_params(12).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = mlp.loss_and_grad(p, X, t)[0]
    for k in range(1, 301):
        L, g = mlp.loss_and_grad(p, X, t)
        p, m, v = mlp.adam_step(p, g, m, v, k, lr=3e-3)
    assert mlp.loss_and_grad(p, X, t)[0] < 0.05 * L0
