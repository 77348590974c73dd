"""Pins of the MLP reference (oracle/mlp.py) against facts outside it:
central finite differences of the loss, scikit-learn's MLP forward pass with
the same weights, Adam's closed-form first step, and exact zero gradients
where ReLU units are dead."""
import numpy as np
import pytest

from oracle import mlp

RNG = np.random.default_rng(0)


def rand_theta(scale=0.3):
    return RNG.normal(0, scale, mlp.N_PARAMS)


def test_param_count():
    assert mlp.N_PARAMS == 24 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5825


def test_gradient_matches_central_differences():
    X = RNG.normal(size=(37, 24))
    t = RNG.normal(size=37)
    th = rand_theta()
    g = mlp.grad(th, X, t)
    h = 1e-6
    idx = RNG.choice(mlp.N_PARAMS, 200, replace=False)
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss(th + e, X, t) - mlp.loss(th - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), i


def test_forward_matches_sklearn():
    from sklearn.neural_network import MLPRegressor
    X = RNG.normal(size=(50, 24))
    th = rand_theta()
    p = mlp.unpack(th)
    reg = MLPRegressor(hidden_layer_sizes=(64, 64), activation="relu", max_iter=1)
    with pytest.warns(Warning):
        reg.fit(X[:5], np.zeros(5))  # creates the arrays; weights are replaced below
    reg.coefs_ = [p["W1"].T.copy(), p["W2"].T.copy(), p["w3"].reshape(64, 1).copy()]
    reg.intercepts_ = [p["b1"].copy(), p["b2"].copy(), p["b3"].copy()]
    np.testing.assert_allclose(mlp.forward(th, X)[0], reg.predict(X), rtol=1e-12, atol=1e-12)


def test_adam_first_step_closed_form():
    # with zero moments, the bias-corrected first step is -lr * g / (|g| + eps)
    th = rand_theta()
    g = RNG.normal(size=mlp.N_PARAMS)
    new, m, v = mlp.adam_step(th, np.zeros_like(th), np.zeros_like(th), g, 1, 1e-3)
    np.testing.assert_allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_dead_relu_units_get_no_gradient():
    X = RNG.normal(size=(20, 24))
    th = rand_theta()
    p = mlp.unpack(th)
    p["b1"][:8] = -1e6  # first 8 hidden units never fire
    th = mlp.pack(p)
    g = mlp.unpack(mlp.grad(th, X, RNG.normal(size=20)))
    assert np.all(g["W1"][:8] == 0) and np.all(g["b1"][:8] == 0) and np.all(g["W2"][:, :8] == 0)


def test_training_reduces_loss_on_a_learnable_target():
    X = RNG.normal(size=(200, 24))
    t = X[:, 0] * 0.5 - X[:, 3] ** 2 * 0.1
    th0 = rand_theta(0.1)
    th, mean, std, hist = mlp.train(th0, X, t, 300, 1e-2)
    assert hist[-1] < 0.2 * hist[0]
    np.testing.assert_allclose(mlp.predict(th, mean, std, X[:5]), mlp.forward(th, (X[:5] - mean) / std)[0])
