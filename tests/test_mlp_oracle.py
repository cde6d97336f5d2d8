"""Pins of the estimator's FP64 oracle: backpropagation against central
differences, a single linear layer against the closed-form gradient
(2/n) X^T (X w - y), and Adam against a hand-stepped first update."""
import numpy as np
import pytest

from oracle import mlp


def _data(n=40, d=6, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, d)), rng.standard_normal(n)


def test_backprop_matches_central_differences():
    X, t = _data()
    p = mlp.init(6, 8, seed=1)
    # keep every pre-activation away from the kink so differences are smooth
    for k in ("b1", "b2"):
        p[k] = p[k] + 0.3
    _, g = mlp.loss_and_grad(p, X, t)
    v = mlp.flatten(p)
    gv = mlp.flatten(g)
    h = 1e-6
    num = np.zeros_like(v)
    for i in range(len(v)):
        e = np.zeros_like(v)
        e[i] = h
        lp, _ = mlp.loss_and_grad(mlp.unflatten(v + e, 6, 8), X, t)
        lm, _ = mlp.loss_and_grad(mlp.unflatten(v - e, 6, 8), X, t)
        num[i] = (lp - lm) / (2 * h)
    assert np.linalg.norm(num - gv) <= 1e-6 * max(1.0, np.linalg.norm(gv))


def test_linear_layer_closed_form():
    # a network whose hidden layers pass positive inputs through (identity
    # weights, inputs shifted positive) is the linear map x -> x w3 + b3
    X, t = _data(n=30, d=4, seed=2)
    X = np.abs(X) + 0.1
    p = mlp.init(4, 4, seed=3)
    p["W1"], p["W2"] = np.eye(4), np.eye(4)
    p["b1"], p["b2"] = np.zeros(4), np.zeros(4)
    p["b3"] = np.array([0.25])
    _, g = mlp.loss_and_grad(p, X, t)
    r = X @ p["w3"] + 0.25 - t
    np.testing.assert_allclose(g["w3"], 2.0 / len(X) * X.T @ r, rtol=1e-12)
    assert g["b3"][0] == pytest.approx(2.0 / len(X) * r.sum(), rel=1e-12)


def test_adam_first_step_is_sign_times_lr():
    # at t = 1 the bias-corrected ratio m/sqrt(v) is g/|g|
    X, t = _data()
    p = mlp.init(6, 8, seed=4)
    _, g = mlp.loss_and_grad(p, X, t)
    before = {k: v.copy() for k, v in p.items()}
    mlp.adam_step(p, g, {}, lr=0.01, eps=0.0)
    for k in mlp.ORDER:
        nz = g[k] != 0
        np.testing.assert_allclose((before[k] - p[k])[nz], 0.01 * np.sign(g[k][nz]), rtol=1e-12)


def test_training_fits_a_smooth_target():
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (256, 3))
    t = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2]
    p = mlp.init(3, 32, seed=6)
    st = {}
    l0, _ = mlp.loss_and_grad(p, X, t)
    for _ in range(2000):
        _, g = mlp.loss_and_grad(p, X, t)
        mlp.adam_step(p, g, st, lr=3e-3)
    l1, _ = mlp.loss_and_grad(p, X, t)
    assert l1 < 0.05 * l0
