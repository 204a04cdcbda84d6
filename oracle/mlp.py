"""FP64 reference MLP (forward, backward, MSE, Adam). TEST INFRASTRUCTURE (oracle).

Not from the paper: the learned band tail replaces the paper's extrapolar
terminator (Eq. X_term_def) by a small network. The network is
X -> [Linear -> SiLU] x L -> Linear, weights W_l stored [out][in] row-major so
that z = h W^T + b. Loss = mean over samples and outputs of (y - t)^2.
Adam follows Kingma & Ba (2015) with bias correction.
Pinned by central finite differences in the test-suite.
"""

from __future__ import annotations

import numpy as np


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * _sig(z)


def silu_grad(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def init_params(dims, seed):
    """He-uniform style init: W_l ~ U(-a, a), a = sqrt(6 / fan_in); b = 0."""
    g = np.random.default_rng(seed)
    params = []
    for din, dout in zip(dims[:-1], dims[1:]):
        a = np.sqrt(6.0 / din)
        params.append((g.uniform(-a, a, (dout, din)), np.zeros(dout)))
    return params


def forward(params, X):
    """Returns the output and the cache of pre-activations/activations."""
    h = np.asarray(X, np.float64)
    hs, zs = [h], []
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        zs.append(z)
        h = silu(z) if li < len(params) - 1 else z
        hs.append(h)
    return h, (hs, zs)


def mse(Y, T):
    d = Y - T
    return float(np.mean(d * d))


def backward(params, cache, Y, T):
    """Gradients of the MSE loss: list of (dW, db), plus dX."""
    hs, zs = cache
    n_el = Y.size
    g = 2.0 * (Y - T) / n_el
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        if li < len(params) - 1:
            g = g * silu_grad(zs[li])
        grads[li] = (g.T @ hs[li], g.sum(axis=0))
        g = g @ W
    return grads, g


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place Adam update; state = dict(t, m, v)."""
    if not state:
        state.update(t=0, m=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params],
                     v=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params])
    state["t"] += 1
    t = state["t"]
    out = []
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        mW, mb = state["m"][i]
        vW, vb = state["v"][i]
        mW = b1 * mW + (1 - b1) * gW
        mb = b1 * mb + (1 - b1) * gb
        vW = b2 * vW + (1 - b2) * gW * gW
        vb = b2 * vb + (1 - b2) * gb * gb
        state["m"][i] = (mW, mb)
        state["v"][i] = (vW, vb)
        c1, c2 = 1 - b1 ** t, 1 - b2 ** t
        W = W - lr * (mW / c1) / (np.sqrt(vW / c2) + eps)
        b = b - lr * (mb / c1) / (np.sqrt(vb / c2) + eps)
        out.append((W, b))
    return out
