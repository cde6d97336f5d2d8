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


def _unit_params(val):
    return {k: np.full(sh, val, dtype=np.float64) for k, sh in
            (("W1", (1, 1)), ("b1", (1,)), ("W2", (1, 1)), ("b2", (1,)), ("w3", (1,)), ("b3", (1,)))}


def test_adam_steps_two_and_three_hand_computed():
    # gradients +g, -g, +g on every parameter (beta1 = 0.9, beta2 = 0.999,
    # eps = 0).  By hand:
    #   t=1: m = 0.1 g,               v = 0.001 g^2,
    #        m/(1-0.9)   = g,          v/(1-0.999)   = g^2     -> step  lr
    #   t=2: m = 0.09 g - 0.1 g = -0.01 g,   v = 0.000999 g^2 + 0.001 g^2 = 0.001999 g^2
    #        m/(1-0.81)  = -g/19,      v/(1-0.998001) = g^2    -> step -lr/19
    #   t=3: m = -0.009 g + 0.1 g = 0.091 g, v = 0.001997001 g^2 + 0.001 g^2 = 0.002997001 g^2
    #        m/(1-0.729) = 91 g/271,   v/(1-0.997002999) = g^2 -> step 91 lr/271
    # (steps are in the direction of sign(g) and are subtracted).
    lr, g0 = 0.01, 0.37
    p = _unit_params(1.0)
    st = {}
    want = 1.0
    for t, (sgn, step) in enumerate(((1, 1.0), (-1, -1.0 / 19.0), (1, 91.0 / 271.0)), start=1):
        g = _unit_params(sgn * g0)
        mlp.adam_step(p, g, st, lr=lr, eps=0.0)
        want -= lr * step
        for k in mlp.ORDER:
            np.testing.assert_allclose(p[k], want, rtol=0, atol=1e-15, err_msg=f"t={t} {k}")
    assert st["t"] == 3


def test_adam_constant_gradient_moves_lr_per_step():
    # with a constant gradient the bias-corrected moments equal g and g^2 at
    # every t, so each step is exactly lr * sign(g); a bias correction with a
    # wrong t, or moments not carried over, breaks this from t = 2 on
    p = _unit_params(0.0)
    st = {}
    for t in range(1, 6):
        mlp.adam_step(p, _unit_params(-2.5), st, lr=0.125, eps=0.0)
        for k in mlp.ORDER:
            np.testing.assert_allclose(p[k], 0.125 * t, rtol=1e-13)


def test_planted_adam_without_moment_carry_is_caught(monkeypatch):
    real = mlp.adam_step

    def forgetful(p, g, state, **kw):   # moments reset every step
        for k in list(state):
            if k != "t":
                del state[k]
        return real(p, g, state, **kw)

    p = _unit_params(1.0)
    st = {}
    for sgn in (1, -1):
        forgetful(p, _unit_params(sgn * 0.37), st, lr=0.01, eps=0.0)
    assert not np.allclose(p["W1"], 1.0 - 0.01 + 0.01 / 19.0, rtol=0, atol=1e-15)


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
