"""Pins of the ridge-regression oracle (section 3, linear regression):
the covariance matrix against the query oracle, the closed-form minimiser
against scikit-learn's ridge solver, the step size against numpy's symmetric
eigensolver, and gradient descent against the closed form."""
import numpy as np
import pytest

import oracle
from oracle import ridge
import workloads as W

CONT = ["units", "i1", "s1", "d1", "w1"]
CATS = ["icat2", "scat2", "wcat1"]


@pytest.fixture(scope="module")
def prob():
    return W.retail_snowflake(seed=3, n_inv=3_000, n_locn=20, n_dates=6, n_ksn=40, n_weather_dates=8,
                              dtype="f64")


@pytest.fixture(scope="module")
def S(prob):
    return ridge.sigma(prob, CONT, CATS)


def test_sigma_closed_forms(prob, S):
    # COUNT = |D| = fact rows (complete foreign keys); Sigma symmetric
    assert S[0, 0] == 3_000
    np.testing.assert_array_equal(S, S.T)
    # one-hot blocks partition D: each block's rows sum to the intercept row
    off = 1 + len(CONT)
    dom = {"icat2": 8, "scat2": 4, "wcat1": 3}
    for c in CATS:
        blk = S[off:off + dom[c]]
        np.testing.assert_allclose(blk.sum(axis=0), S[0], rtol=1e-12, atol=1e-9)
        # a tuple has one code: off-diagonal entries inside a block vanish
        inner = S[off:off + dom[c], off:off + dom[c]]
        np.testing.assert_array_equal(inner, np.diag(np.diag(inner)))
        off += dom[c]


def test_sigma_matches_query_oracle(prob, S):
    # the same entries computed as aggregate queries over D
    qs = [{"groupby": [], "where": [], "aggs": [[("units", 1), ("s1", 1)]], "root": None},
          {"groupby": ["scat2"], "where": [], "aggs": [[("w1", 1)]], "root": None},
          {"groupby": ["icat2", "wcat1"], "where": [], "aggs": [[]], "root": None}]
    r = oracle.evaluate(dict(prob, batch=qs))
    i_units, i_s1, i_w1 = 1 + CONT.index("units"), 1 + CONT.index("s1"), 1 + CONT.index("w1")
    assert S[i_units, i_s1] == pytest.approx(float(r[0]["sum"][0, 0]), rel=1e-12)
    off_scat2 = 1 + len(CONT) + 8
    for k, v in zip(r[1]["keys"][:, 0], r[1]["sum"][:, 0]):
        assert S[off_scat2 + k, i_w1] == pytest.approx(float(v), rel=1e-12, abs=1e-9)
    off_icat2, off_wcat1 = 1 + len(CONT), 1 + len(CONT) + 8 + 4
    for (a, b), c in zip(r[2]["keys"], r[2]["count"]):
        assert S[off_icat2 + a, off_wcat1 + b] == c


def test_closed_form_matches_sklearn(prob, S):
    from sklearn.linear_model import Ridge
    label, lam = 1 + CONT.index("units"), 0.05
    theta = ridge.closed_form(S, label, lam)
    X = ridge.design_matrix(prob, CONT, CATS)
    F = [i for i in range(X.shape[1]) if i != label]
    # J = ||X_F theta_F - y||^2 / (2n) + lam/2 ||theta_F||^2  <=>  sklearn alpha = n * lam
    m = Ridge(alpha=len(X) * lam, fit_intercept=False, solver="cholesky", tol=1e-14).fit(X[:, F], X[:, label])
    np.testing.assert_allclose(theta[F], m.coef_, rtol=1e-7, atol=1e-10)
    assert theta[label] == -1.0


def test_power_step_is_inverse_top_eigenvalue(S):
    label, lam = 1, 0.05
    F = [i for i in range(len(S)) if i != label]
    A = S[np.ix_(F, F)] / S[0, 0] + lam * np.eye(len(F))
    L = np.linalg.eigvalsh(A).max()
    assert ridge.power_step(S, label, lam, iters=500) == pytest.approx(1.0 / L, rel=1e-9)


def test_bgd_converges_to_closed_form(S):
    label, lam = 1, 0.5
    eta = ridge.power_step(S, label, lam, iters=500)
    theta, steps, gn = ridge.bgd(S, label, lam, eta, iters=200_000, tol=1e-11)
    assert gn <= 1e-11 and steps < 200_000
    np.testing.assert_allclose(theta, ridge.closed_form(S, label, lam), rtol=0, atol=1e-8)


def test_planted_sign_error_is_caught(S):
    # a gradient with the wrong sign on the regulariser does not reach the minimiser
    label, lam = 1, 0.5
    F = np.array([i for i in range(len(S)) if i != label])
    eta = ridge.power_step(S, label, lam)
    theta = np.zeros(len(S))
    theta[label] = -1.0
    for _ in range(3000):
        g = (S @ theta)[F] / S[0, 0] - lam * theta[F]
        theta[F] -= eta * g
    assert np.abs(theta - ridge.closed_form(S, label, lam)).max() > 1e-6
