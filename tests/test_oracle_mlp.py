"""Pins of the reference MLP: central finite differences and an Adam closed form."""

import numpy as np

from oracle import mlp


def test_mlp_gradients_vs_central_differences():
    dims = [5, 7, 6, 2]
    params = mlp.init_params(dims, 3)
    g = np.random.default_rng(1)
    X = g.normal(size=(9, 5))
    T = g.normal(size=(9, 2))
    Y, cache = mlp.forward(params, X)
    grads, dX = mlp.backward(params, cache, Y, T)
    h = 1e-6

    def loss(ps, x=X):
        return mlp.mse(mlp.forward(ps, x)[0], T)

    for li in range(len(params)):
        W, b = params[li]
        for (i, j) in [(0, 0), (1, 2), (W.shape[0] - 1, W.shape[1] - 1)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[i, j] += h
            Wm[i, j] -= h
            pp = list(params); pp[li] = (Wp, b)
            pm = list(params); pm[li] = (Wm, b)
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(fd - grads[li][0][i, j]) <= 1e-6 * max(1e-3, abs(fd))
        for i in range(b.shape[0]):
            bp, bm = b.copy(), b.copy()
            bp[i] += h
            bm[i] -= h
            pp = list(params); pp[li] = (W, bp)
            pm = list(params); pm[li] = (W, bm)
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(fd - grads[li][1][i]) <= 1e-6 * max(1e-3, abs(fd))
    for (i, j) in [(0, 0), (4, 3)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[i, j] += h
        Xm[i, j] -= h
        fd = (loss(params, Xp) - loss(params, Xm)) / (2 * h)
        assert abs(fd - dX[i, j]) <= 1e-6 * max(1e-3, abs(fd))


def test_silu_values():
    assert mlp.silu(np.array(0.0)) == 0.0
    assert abs(mlp.silu(np.array(2.0)) - 2.0 / (1.0 + np.exp(-2.0))) < 1e-15
    z = np.linspace(-4, 4, 9)
    fd = (mlp.silu(z + 1e-6) - mlp.silu(z - 1e-6)) / 2e-6
    assert np.abs(fd - mlp.silu_grad(z)).max() < 1e-8


def test_adam_first_step_is_signed_lr():
    # after one step with bias correction, the update is lr * g / (|g| + eps)
    params = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[0.3, -4.0]]), np.array([1e-3]))]
    st = {}
    out = mlp.adam_step(params, grads, st, lr=0.1)
    assert np.allclose(out[0][0], [[1.0 - 0.1, -2.0 + 0.1]], atol=1e-6)
    assert np.allclose(out[0][1], [0.5 - 0.1 * 1e-3 / (1e-3 + 1e-8)])


def test_training_reduces_loss():
    g = np.random.default_rng(0)
    X = g.normal(size=(64, 3))
    T = np.stack([np.sin(X[:, 0]) + X[:, 1] * X[:, 2], X[:, 0] ** 2], 1)
    params = mlp.init_params([3, 32, 32, 2], 0)
    st = {}
    l0 = mlp.mse(mlp.forward(params, X)[0], T)
    for _ in range(300):
        Y, c = mlp.forward(params, X)
        gr, _ = mlp.backward(params, c, Y, T)
        params = mlp.adam_step(params, gr, st, lr=3e-3)
    assert mlp.mse(mlp.forward(params, X)[0], T) < 0.1 * l0
