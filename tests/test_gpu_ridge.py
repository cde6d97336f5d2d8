"""Ridge regression on the GPU (section 3, linear regression): the
covariance matrix assembled from the batch's results against the oracle's
X^T X, gradient descent against the oracle's iteration on the same matrix,
and convergence to the closed-form minimiser."""
import numpy as np
import pytest

from oracle import ridge
import workloads as W

pytestmark = pytest.mark.gpu

CONT = ["units", "i1", "i2", "s1", "s2", "d1", "w1", "w2"]
CATS = ["icat1", "scat1", "wcat2"]


@pytest.fixture(scope="module")
def run():
    import torch
    assert torch.cuda.is_available()
    import paper_2008_08657_amd as E
    p = W.retail_snowflake(seed=5, n_inv=60_000, n_locn=30, n_dates=10, n_ksn=200, n_weather_dates=12,
                           dtype="f64")
    p["batch"] = W.covariance_batch(CONT, CATS)
    plan = E.Plan(p, precision="f64", policy="fact", row_piece_max=5_000, min_segment=16)
    prep = E.Prepared(plan, E.device_columns(p))
    prep.run(sync=True)
    return E, p, prep


def test_sigma_matches_design_matrix(run):
    E, p, prep = run
    got = prep.ridge_sigma(CONT, CATS).cpu().numpy()
    X = ridge.design_matrix(p, CONT, CATS)
    ref = X.T @ X
    absr = np.abs(X).T @ np.abs(X)
    assert got.shape == ref.shape
    scale = np.maximum(np.abs(ref), 1e-3 * absr)
    scale[scale == 0] = 1.0
    assert np.max(np.abs(got - ref) / scale) <= 1e-12
    np.testing.assert_array_equal(got, got.T)


def test_bgd_steps_match_oracle(run):
    E, p, prep = run
    sig = prep.ridge_sigma(CONT, CATS)
    S = sig.cpu().numpy()
    label, lam = 1, 0.01
    eta = ridge.power_step(S, label, lam)
    for k in (1, 7, 100):
        th, steps, gn, used = E.ridge_bgd(sig, label, lam, eta=eta, max_iter=k, tol=0.0)
        ref, rsteps, rgn = ridge.bgd(S, label, lam, eta, iters=k)
        assert steps == rsteps == k and used == eta
        t = th.cpu().numpy()
        assert np.linalg.norm(t - ref) <= 1e-12 * np.linalg.norm(ref)
        assert gn == pytest.approx(rgn, rel=1e-10)


def test_bgd_step_size_and_convergence(run):
    E, p, prep = run
    sig = prep.ridge_sigma(CONT, CATS)
    S = sig.cpu().numpy()
    label, lam = 1, 0.5
    th, steps, gn, eta = E.ridge_bgd(sig, label, lam, eta=0.0, max_iter=200_000, tol=1e-11)
    assert eta == pytest.approx(ridge.power_step(S, label, lam), rel=1e-12)
    assert gn <= 1e-11 and steps < 200_000
    np.testing.assert_allclose(th.cpu().numpy(), ridge.closed_form(S, label, lam), rtol=0, atol=1e-8)
