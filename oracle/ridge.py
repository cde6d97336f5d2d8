"""Ridge linear regression by batch gradient descent over the covariance
matrix (paper, section 3, "Linear Regression").

TEST INFRASTRUCTURE ONLY (same rules as the ``oracle`` package).

The model is LR(x) = <theta, x> with x_1 = 1 (the intercept) and the label
inside x with its parameter fixed to -1.  With Sigma = sum over D of x x^T
(categoricals one-hot encoded), the objective and gradient are

    J(theta)      = theta^T Sigma theta / (2 |D|) + lambda/2 ||theta||^2
    grad J(theta) = Sigma theta / |D| + lambda theta,

taken over the free parameters only (every entry except the label's).
Readings where the paper is silent: every free parameter, the intercept
included, is regularised; the step size is eta = 1/L with L the largest
eigenvalue of Sigma_FF/|D| + lambda I, found by power iteration; theta starts
at 0 on the free entries.

Layout of x (and of Sigma): index 0 the intercept, then the continuous
attributes in the order given, then for every categorical attribute its
one-hot block over its whole domain [0, domain).
"""
from __future__ import annotations

import numpy as np

from . import materialize_join

__all__ = ["design_matrix", "sigma", "power_step", "bgd", "closed_form"]


def design_matrix(problem: dict, continuous, categorical) -> np.ndarray:
    """x for every tuple of the materialised join D, FP64 (section 3: one-hot
    encoding of categorical attributes)."""
    D = materialize_join(problem, list(continuous) + list(categorical))
    n = len(D[continuous[0]]) if continuous else len(D[categorical[0]])
    dom = {a["name"]: a["domain"] for r in problem["schema"] for a in r["attrs"]}
    cols = [np.ones(n)]
    cols += [np.asarray(D[c], dtype=np.float64) for c in continuous]
    for c in categorical:
        onehot = np.zeros((n, dom[c]))
        onehot[np.arange(n), np.asarray(D[c], dtype=np.int64)] = 1.0
        cols.append(onehot)
    return np.column_stack(cols)


def sigma(problem: dict, continuous, categorical) -> np.ndarray:
    """Sigma = sum over D of x x^T (the non-centred covariance matrix)."""
    X = design_matrix(problem, continuous, categorical)
    return X.T @ X


def _free(dim: int, label: int) -> np.ndarray:
    return np.array([i for i in range(dim) if i != label])


def power_step(S: np.ndarray, label: int, lam: float, iters: int = 100) -> float:
    """eta = 1/L, L = largest eigenvalue of Sigma_FF/|D| + lambda I, by power
    iteration from the all-ones vector (Rayleigh quotient of the last iterate)."""
    n = S[0, 0]
    F = _free(len(S), label)
    A = S[np.ix_(F, F)] / n + lam * np.eye(len(F))
    v = np.ones(len(F)) / np.sqrt(len(F))
    for _ in range(iters):
        w = A @ v
        v = w / np.linalg.norm(w)
    return 1.0 / float(v @ (A @ v))


def bgd(S: np.ndarray, label: int, lam: float, eta: float, iters: int, tol: float = 0.0):
    """Batch gradient descent: theta_F <- theta_F - eta * grad_F J, the label's
    parameter held at -1.  Stops after ``iters`` steps or when ||grad_F|| <=
    tol.  Returns (theta, steps taken, ||grad_F|| at the last iterate)."""
    n = S[0, 0]
    dim = len(S)
    F = _free(dim, label)
    theta = np.zeros(dim)
    theta[label] = -1.0
    steps = 0
    while True:
        g = (S @ theta)[F] / n + lam * theta[F]
        gn = float(np.linalg.norm(g))
        if gn <= tol or steps >= iters:
            return theta, steps, gn
        theta[F] -= eta * g
        steps += 1


def closed_form(S: np.ndarray, label: int, lam: float) -> np.ndarray:
    """The minimiser: grad_F J = 0 gives (Sigma_FF/|D| + lambda I) theta_F =
    Sigma_F,label/|D| (theta_label = -1)."""
    n = S[0, 0]
    dim = len(S)
    F = _free(dim, label)
    A = S[np.ix_(F, F)] / n + lam * np.eye(len(F))
    theta = np.zeros(dim)
    theta[label] = -1.0
    theta[F] = np.linalg.solve(A, S[F, label] / n)
    return theta
