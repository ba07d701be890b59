"""Pins of the FP64 warm-start network oracle."""
import numpy as np

import scenes
from oracle import mlp


def _params(seed=0):
    p = scenes.mlp_init(6, 5, 4, seed)
    return {k: v.astype(np.float64) for k, v in p.items()}


def test_silu_derivative_closed_form():
    t = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(t + h) - mlp.silu(t - h)) / (2 * h)
    assert np.abs(fd - mlp.silu_grad(t)).max() <= 1e-8
    assert mlp.silu(0.0) == 0.0 and mlp.silu_grad(0.0) == 0.5


def test_backward_matches_finite_differences():
    p = _params(1)
    rng = np.random.default_rng(2)
    Z = rng.standard_normal((7, 6))
    T = rng.standard_normal((7, 4))
    Y, cache = mlp.forward(p, Z)
    g = mlp.backward(p, cache, Y, T)
    h = 1e-6
    for k in p:
        flat = p[k].ravel()
        for j in range(0, flat.size, max(1, flat.size // 7)):
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k].ravel()[j] += h
            lp = mlp.loss(mlp.forward(q, Z)[0], T)
            q[k].ravel()[j] -= 2 * h
            lm = mlp.loss(mlp.forward(q, Z)[0], T)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].ravel()[j]) <= 1e-7 * max(1.0, abs(fd)), (k, j)


def test_adam_first_step_and_quadratic():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -1e-3, 2.0])}
    st = mlp.adam_init(p)
    q = mlp.adam_step(p, g, st, lr=0.1)
    # bias-corrected first step: -lr * g / (|g| + eps)
    assert np.allclose(q["w"] - p["w"], -0.1 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=1e-12, atol=0)
    # minimises a convex quadratic
    c = np.array([0.3, -0.7, 1.1])
    st = mlp.adam_init(p)
    for _ in range(3000):
        p = mlp.adam_step(p, {"w": 2 * (p["w"] - c)}, st, lr=0.01)
    assert np.abs(p["w"] - c).max() <= 1e-3


def test_training_reduces_the_loss_on_a_learnable_map():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((256, 6))
    Y = np.tanh(X[:, :4] * 0.5)
    p0 = scenes.mlp_init(6, 16, 4, 3)
    order = scenes.minibatch_order(256, 32, 300, seed=5)
    _, losses = mlp.train(p0, X, Y, order, lr=3e-3)
    assert np.mean(losses[-20:]) < 0.2 * np.mean(losses[:5])
