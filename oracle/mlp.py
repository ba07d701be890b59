"""The warm-start network in FP64 (CPU oracle).  Test infrastructure only.

Not part of the paper: a three-layer perceptron maps the last two coarse
states (standardised) to a correction of the constant-velocity prediction of
the next one:
    h0 = W0 z + b0,  a0 = silu(h0),
    h1 = W1 a0 + b1, a1 = silu(h1),
    y  = W2 a1 + b2,                 silu(t) = t / (1 + exp(-t)),
trained on the mean squared error L = mean((y - t)^2) over a minibatch and
all outputs with Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).

Pinned by tests/test_oracle_mlp.py: central finite differences of the loss
against the hand-written backward pass, the closed form of silu', and
Adam's first step (-lr sign(g)) and a quadratic it must minimise.
"""
from __future__ import annotations

import numpy as np


def silu(t):
    return t / (1.0 + np.exp(-t))


def silu_grad(t):
    s = 1.0 / (1.0 + np.exp(-t))
    return s * (1.0 + t * (1.0 - s))


def forward(p, Z):
    """Z [B, in] -> (Y [B, out], cache)."""
    Z = np.asarray(Z, dtype=np.float64)
    h0 = Z @ p["W0"].T + p["b0"]
    a0 = silu(h0)
    h1 = a0 @ p["W1"].T + p["b1"]
    a1 = silu(h1)
    y = a1 @ p["W2"].T + p["b2"]
    return y, (Z, h0, a0, h1, a1)


def loss(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(p, cache, Y, T):
    """Gradients of mean((Y - T)^2) with respect to every parameter."""
    Z, h0, a0, h1, a1 = cache
    dY = 2.0 * (Y - T) / Y.size
    g = {"W2": dY.T @ a1, "b2": dY.sum(axis=0)}
    dh1 = (dY @ p["W2"]) * silu_grad(h1)
    g["W1"] = dh1.T @ a0
    g["b1"] = dh1.sum(axis=0)
    dh0 = (dh1 @ p["W1"]) * silu_grad(h0)
    g["W0"] = dh0.T @ Z
    g["b0"] = dh0.sum(axis=0)
    return g


def adam_init(p):
    return {"t": 0, "m": {k: np.zeros_like(v, dtype=np.float64) for k, v in p.items()},
            "v": {k: np.zeros_like(v, dtype=np.float64) for k, v in p.items()}}


def adam_step(p, g, st, lr, b1=0.9, b2=0.999, eps=1e-8):
    st["t"] += 1
    t = st["t"]
    out = {}
    for k in p:
        st["m"][k] = b1 * st["m"][k] + (1 - b1) * g[k]
        st["v"][k] = b2 * st["v"][k] + (1 - b2) * g[k] ** 2
        mh = st["m"][k] / (1 - b1 ** t)
        vh = st["v"][k] / (1 - b2 ** t)
        out[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return out


def train(p, X, Y, order, lr):
    """Adam over the minibatches order[s] (indices into X, Y); returns the
    parameters and the loss of every step (before its update)."""
    p = {k: np.asarray(v, dtype=np.float64) for k, v in p.items()}
    st = adam_init(p)
    losses = []
    for idx in order:
        Yh, cache = forward(p, X[idx])
        losses.append(loss(Yh, Y[idx]))
        p = adam_step(p, backward(p, cache, Yh, Y[idx]), st, lr)
    return p, losses
