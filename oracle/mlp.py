"""Multilayer-perceptron estimator of group counts: forward pass, gradient of
the mean squared error, and Adam steps, in FP64.

TEST INFRASTRUCTURE ONLY (same rules as the ``oracle`` package).

Network: x (d features) -> h1 = relu(x W1 + b1) -> h2 = relu(h1 W2 + b2)
-> y = h2 w3 + b3, one output.  Loss: mean over the batch of (y - t)^2.
Adam (Kingma and Ba, 2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parameters are a dict of arrays: W1 (d x h), b1 (h), W2 (h x h), b2 (h),
w3 (h), b3 (scalar as a 1-array).
"""
from __future__ import annotations

import numpy as np

__all__ = ["init", "forward", "loss_and_grad", "adam_step", "flatten", "unflatten"]

ORDER = ["W1", "b1", "W2", "b2", "w3", "b3"]


def init(d: int, h: int, seed: int) -> dict:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; numpy PCG64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return {"W1": rng.standard_normal((d, h)) * np.sqrt(2.0 / d), "b1": np.zeros(h),
            "W2": rng.standard_normal((h, h)) * np.sqrt(2.0 / h), "b2": np.zeros(h),
            "w3": rng.standard_normal(h) * np.sqrt(2.0 / h), "b3": np.zeros(1)}


def forward(p: dict, X: np.ndarray):
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (z1, h1, z2, h2)


def loss_and_grad(p: dict, X: np.ndarray, t: np.ndarray):
    """Mean squared error and its gradient by the chain rule."""
    n = len(X)
    y, (z1, h1, z2, h2) = forward(p, X)
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dh2 = np.outer(dy, p["w3"]) * (z2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"].T) * (z1 > 0)
    g["W1"] = X.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return loss, g


def adam_step(p: dict, g: dict, state: dict, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8) -> None:
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in ORDER:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] * g[k]
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def flatten(p: dict) -> np.ndarray:
    """Parameters in the order W1 (row-major), b1, W2, b2, w3, b3."""
    return np.concatenate([np.ravel(p[k]) for k in ORDER])


def unflatten(v: np.ndarray, d: int, h: int) -> dict:
    sizes = {"W1": (d, h), "b1": (h,), "W2": (h, h), "b2": (h,), "w3": (h,), "b3": (1,)}
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(sizes[k]))
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(sizes[k])
        o += n
    return out
