"""The estimator network's GPU kernels against the FP64 oracle
(``oracle.mlp``): forward outputs, backpropagated gradients and Adam steps,
through the C ABI; plus a training run that must lower the loss."""
import numpy as np
import pytest

from oracle import mlp
import paper_2008_08657_amd as lm

D, H = 12, 32


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, D))
    # a smooth target the network can fit: a few products and a log
    t = 0.7 * X[:, 0] * X[:, 1] - 0.3 * X[:, 2] + np.log1p(X[:, 3] ** 2) + 0.1 * rng.standard_normal(n)
    return X, t


def _dev(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype or np.float32)).to("cuda:0")


def test_size_and_argument_checks():
    assert lm.mlp_size(D, H) == D * H + H + H * H + H + H + 1
    lib = lm.load_library()
    assert lib.lmfao_mlp_grad(0, H, None, None, None, 1, None, None, None) == 1


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 37, 300])
def test_forward_and_gradient_parity(n):
    X, t = _problem(n, seed=10 + n)
    p = mlp.init(D, H, seed=3)
    for k in ("b1", "b2"):
        p[k] = p[k] + 0.05
    # FP32 parameters, so both sides start from the same values
    v32 = mlp.flatten(p).astype(np.float32)
    p64 = mlp.unflatten(v32.astype(np.float64), D, H)
    X32 = X.astype(np.float32)
    t32 = t.astype(np.float32)
    loss_o, g_o = mlp.loss_and_grad(p64, X32.astype(np.float64), t32.astype(np.float64))
    y_o, _ = mlp.forward(p64, X32.astype(np.float64))
    y = lm.mlp_predict(_dev(v32), _dev(X32), H).cpu().numpy()
    np.testing.assert_allclose(y, y_o, rtol=1e-4, atol=1e-4 * max(1.0, np.abs(y_o).max()))
    g, loss = lm.mlp_grad(_dev(v32), _dev(X32), _dev(t32), H)
    g = g.cpu().numpy().astype(np.float64)
    go = mlp.flatten(g_o)
    assert loss == pytest.approx(loss_o, rel=1e-4)
    # FP32 accumulation over n rows of unit-scale terms
    assert np.linalg.norm(g - go) <= 1e-4 * max(1e-3, np.linalg.norm(go))


@pytest.mark.gpu
def test_adam_steps_parity():
    import torch
    n, batch, steps, lr = 256, 64, 5, 1e-3
    X, t = _problem(n, seed=5)
    X32, t32 = X.astype(np.float32), t.astype(np.float32)
    v32 = mlp.flatten(mlp.init(D, H, seed=8)).astype(np.float32)
    order = np.random.default_rng(6).integers(0, n, size=steps * batch).astype(np.int32)
    params = _dev(v32)
    trace = lm.mlp_train(params, _dev(X32), _dev(t32), _dev(order, np.int32), batch, H, lr=lr)
    p = mlp.unflatten(v32.astype(np.float64), D, H)
    state = {}
    gmax = []
    for s in range(steps):
        rows = order[s * batch:(s + 1) * batch]
        loss, g = mlp.loss_and_grad(p, X32[rows].astype(np.float64), t32[rows].astype(np.float64))
        assert trace[s] == pytest.approx(loss, rel=1e-4)
        gmax.append(np.abs(mlp.flatten(g)))
        mlp.adam_step(p, g, state, lr=lr)
    got = params.cpu().numpy().astype(np.float64)
    want = mlp.flatten(p)
    # a component whose gradient is near zero can take a step of either sign
    # in FP32; every other component must follow the FP64 steps closely
    small = np.min(gmax, axis=0) <= 1e-4 * max(g.max() for g in gmax)
    err = np.abs(got - want)
    assert np.all(err[~small] <= 1e-5 + 1e-4 * np.abs(want[~small]))
    assert np.all(err[small] <= 2 * lr * steps + 1e-6)
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_training_lowers_the_loss():
    n, batch, steps = 2048, 128, 400
    X, t = _problem(n, seed=11)
    X32, t32 = X.astype(np.float32), t.astype(np.float32)
    params = _dev(mlp.flatten(mlp.init(D, H, seed=12)).astype(np.float32))
    order = _dev(np.random.default_rng(13).integers(0, n, size=steps * batch).astype(np.int32), np.int32)
    Xd, td = _dev(X32), _dev(t32)
    _, before = lm.mlp_grad(params, Xd, td, H)
    trace = lm.mlp_train(params, Xd, td, order, batch, H, lr=3e-3)
    _, after = lm.mlp_grad(params, Xd, td, H)
    assert np.all(np.isfinite(trace))
    assert after < 0.25 * before
    assert np.mean(trace[-20:]) < np.mean(trace[:20])
