"""GPU warm-start network (bf16 matrix cores, FP32 accumulation) against
the FP64 oracle, and timesteps started from its prediction."""
import numpy as np
import pytest

import scenes
from oracle import fem, mlp, newton
from tests.gpu_util import device, e_rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _abs_bound(p, Z):
    """Propagated absolute sums |W2| 1.1 (|W1| 1.1 (|W0| |z| + |b0|) + |b1|) + |b2|:
    bf16 operands with FP32 accumulation keep each layer's error below a
    small multiple of 2^-8 of these sums (silu' <= 1.1)."""
    a0 = np.abs(Z) @ np.abs(p["W0"]).T + np.abs(p["b0"])
    a1 = 1.1 * a0 @ np.abs(p["W1"]).T + np.abs(p["b1"])
    return 1.1 * a1 @ np.abs(p["W2"]).T + np.abs(p["b2"])


@pytest.mark.parametrize("dims,n", [((40, 32, 20), 5), ((130, 70, 65), 37), ((1032, 256, 516), 3)])
def test_mlp_forward_matches_oracle(dev, dims, n):
    from paper_2508_13386_amd import ms
    i, w, o = dims
    p = scenes.mlp_init(i, w, o, seed=1)
    Z = np.random.default_rng(2).standard_normal((n, i)).astype(np.float32)
    Y = ms.ms_mlp_forward(dev, p, Z)
    p64 = {k: v.astype(np.float64) for k, v in p.items()}
    Yo, _ = mlp.forward(p64, Z.astype(np.float64))
    err = np.abs(Y - Yo) / _abs_bound(p64, Z.astype(np.float64))
    say("mlp forward", dims, n, "max err / bound-scale", err.max())
    assert err.max() <= 3 * 2.0 ** -8


def _grad_scales(p, Z, Y, T):
    """Absolute-value propagation of the backward pass: the same sums as the
    gradients with every operand replaced by an upper bound of its magnitude
    (forward magnitudes as in _abs_bound, |silu| <= |t|, silu' <= 1.1), plus
    the forward error scale in dY.  Each bf16 product contributes at most
    2 * 2^-8 of its absolute value and the deepest gradient passes through
    five rounded products (three forward, two backward), so every entry's
    error stays below 10 * 2^-8 of its scale."""
    h0 = np.abs(Z) @ np.abs(p["W0"]).T + np.abs(p["b0"])
    a0 = 1.1 * h0
    h1 = a0 @ np.abs(p["W1"]).T + np.abs(p["b1"])
    a1 = 1.1 * h1
    yabs = a1 @ np.abs(p["W2"]).T + np.abs(p["b2"])
    dY = 2.0 * (np.abs(Y - T) + yabs) / Y.size
    S = {"W2": dY.T @ a1, "b2": dY.sum(axis=0)}
    dh1 = 1.1 * (dY @ np.abs(p["W2"]))
    S["W1"], S["b1"] = dh1.T @ a0, dh1.sum(axis=0)
    dh0 = 1.1 * (dh1 @ np.abs(p["W1"]))
    S["W0"], S["b0"] = dh0.T @ np.abs(Z), dh0.sum(axis=0)
    return S


def test_mlp_first_gradients_match_oracle(dev):
    """Every gradient entry within the bf16 error bound of its propagated
    absolute scale (elementwise, not through a norm)."""
    from paper_2508_13386_amd import ms
    i, w, o = 72, 48, 36
    p = scenes.mlp_init(i, w, o, seed=3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((100, i)).astype(np.float32)
    T = np.tanh(X[:, :o]).astype(np.float32)
    order = scenes.minibatch_order(100, 32, 1, seed=5)
    lr = 1e-3
    p1, losses, g = ms.ms_mlp_train(dev, p, X, T, order, lr=lr, grads=True)
    p64 = {k: v.astype(np.float64) for k, v in p.items()}
    idx = order[0]
    Z = X[idx].astype(np.float64)
    Yo, cache = mlp.forward(p64, Z)
    go = mlp.backward(p64, cache, Yo, T[idx].astype(np.float64))
    S = _grad_scales(p64, Z, Yo, T[idx].astype(np.float64))
    assert losses[0] == pytest.approx(mlp.loss(Yo, T[idx]), rel=2e-2)
    for k in go:
        err = np.abs(g[k] - go[k]) / S[k]
        say("grad", k, "max err / scale", float(err.max()), "bound", 10 * 2.0 ** -8)
        assert err.max() <= 10 * 2.0 ** -8
        # Adam's first step (bias-corrected m = g, v = g^2) moves each weight
        # by -lr g / (|g| + 1e-8) with the gradient it computed (checked
        # above): about -lr sign(g), in the oracle's direction wherever the
        # GPU gradient's sign is the oracle's; up to float32 rounding
        sure = (np.abs(go[k]) > 2 * np.abs(g[k] - go[k])) & (np.abs(go[k]) > 1e-6)
        say("   adam first step checked on", int(sure.sum()), "of", sure.size)
        if sure.any():
            step = (p1[k] - p[k])[sure].astype(np.float64)
            gk = g[k][sure].astype(np.float64)
            expect = -lr * gk / (np.abs(gk) + 1e-8)
            assert (np.sign(expect) == -np.sign(go[k][sure])).all()
            tol = 1e-5 * lr + 4 * np.finfo(np.float32).eps * np.abs(p[k][sure])
            assert (np.abs(step - expect) <= tol).all()


def test_mlp_training_tracks_oracle(dev):
    from paper_2508_13386_amd import ms
    rng = np.random.default_rng(6)
    X = rng.standard_normal((256, 24)).astype(np.float32)
    T = np.tanh(0.5 * X[:, :12]).astype(np.float32)
    p0 = scenes.mlp_init(24, 32, 12, seed=7)
    order = scenes.minibatch_order(256, 32, 300, seed=8)
    _, lg, _ = ms.ms_mlp_train(dev, p0, X, T, order, lr=3e-3)
    _, lo = mlp.train(p0, X.astype(np.float64), T.astype(np.float64), order, lr=3e-3)
    say("loss gpu", lg[0], lg[-1], "oracle", lo[0], lo[-1])
    assert np.mean(lg[-20:]) < 0.2 * np.mean(lg[:5])
    assert np.mean(lg[-20:]) <= 1.5 * np.mean(lo[-20:]) + 1e-4


def test_warm_started_steps_match_oracle(dev):
    """A network with zero weights predicts the constant-velocity coarse
    state; the step it starts must still land on the oracle's minimiser."""
    from paper_2508_13386_amd import ms
    s = scenes.inclusion_block(8, seed=1, steps=4)
    c = ms.context_from_scene(dev, s)
    c.ms_build_basis(n_handles=8, seed=2)
    r = 12 * c.ms_get_basis()["m"]
    zero = {k: np.zeros_like(v) for k, v in scenes.mlp_init(2 * r, 16, r, seed=0).items()}
    c.ms_set_warmstart(zero, np.zeros(2 * r), np.ones(2 * r), np.ones(r))
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    x, v = s["x0"].copy(), s["v0"].copy()
    used = []
    for k in range(1, 5):
        xo, vo, _ = newton.newton_step(body, x, v, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](k))
        c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        # without the inertial candidate the learned move competes with x^t only
        st = c.ms_step(s["dt"], warm_start=1, predictor=0 if k < 4 else 1)
        xg, vg = c.ms_get_state()
        err = e_rel(xg, xo, x)
        used.append(st["warm_start_used"])
        say("warm step", k, "e_rel", err, "used", st["warm_start_used"], "newton", st["newton_iters"])
        assert err <= 1e-6
        x, v = xg, vg  # continue from the GPU state: the coarse history is the GPU's
    assert used[0] == 0 and sum(used[1:3]) >= 1
    c.close()


def test_trained_warm_start_on_heldout_seeds(dev):
    """What the trained network gains over the method without it, measured on
    held-out trajectories: a network trained on the coarse states of solver
    trajectories (one fixed block, drives varying by seed, one shared basis)
    predicts the next coarse state; each held-out step is run with and
    without it.  Both forms reach the same minimiser at every step; the
    Newton and PCG counts of both and the steps where the learned start was
    taken are reported.  No gain is asserted: on this workload the learned
    coarse start rarely beats the inertial predictor."""
    from paper_2508_13386_amd import ms
    N, steps = 8, 10
    basis = {}
    form = dict(precision=ms.PREC_MIXED, preconditioner=ms.PC_TWO_LEVEL_ADDITIVE, forcing=1, pcg_eta_max=0.1,
                pcg_eta_min=1e-4, coarse_move=0.2, max_newton=100)

    def run(seed, warm=None):
        sc = scenes.learned_drive_scene(seed, N=N, steps=steps)
        c = ms.context_from_scene(dev, sc)
        if not basis:
            c.ms_build_basis(n_handles=8, seed=1)
            basis.update(c.ms_get_basis())
        else:
            c.ms_set_basis(basis["origins"], basis["vptr"], basis["vhandle"], basis["vphi"])
        r = 12 * basis["m"]
        if warm is not None:
            c.ms_set_warmstart(*warm)
        qs, stats, xs = [c.ms_get_coarse(r)], [], []
        for k in range(1, steps + 1):
            c.ms_set_dirichlet(sc["dirichlet"], sc["dbc_targets"](k))
            stats.append(c.ms_step(sc["dt"], ms.solver_defaults(warm_start=1 if warm else 0, **form)))
            qs.append(c.ms_get_coarse(r))
            xs.append(c.ms_get_state()[0])
        c.close()
        return np.array(qs), stats, xs, sc

    train = [run(sd) for sd in scenes.TRAIN_SEEDS[:8]]
    r = 12 * basis["m"]
    X = np.array([np.concatenate([q[k - 1], q[k]]) for q, _, _, _ in train for k in range(1, len(q) - 1)])
    Y = np.array([q[k + 1] - (2 * q[k] - q[k - 1]) for q, _, _, _ in train for k in range(1, len(q) - 1)])
    mean = X.mean(axis=0)
    std = np.full(X.shape[1], (X - mean).std() + 1e-30)
    osc = np.full(Y.shape[1], Y.std() + 1e-30)
    Xn, Yn = ((X - mean) / std).astype(np.float32), (Y / osc).astype(np.float32)
    order = scenes.minibatch_order(len(Xn), 32, 400, seed=1)
    params, losses, _ = ms.ms_mlp_train(dev, scenes.mlp_init(2 * r, 64, r, seed=0), Xn, Yn, order, lr=1e-3)
    say("training samples", len(Xn), "loss", float(np.mean(losses[:20])), "->", float(np.mean(losses[-20:])))
    assert np.mean(losses[-20:]) < np.mean(losses[:20])
    warm = (params, mean, std, osc)
    tot = np.zeros((2, 2), dtype=np.int64)  # [without, with] x [newton, pcg]
    taken = 0
    for sd in scenes.HELDOUT_SEEDS[:2]:
        _, s0, x0, sc = run(sd)
        _, s1, x1, _ = run(sd, warm)
        for k in range(steps):
            u = np.linalg.norm(x0[k] - sc["rest"])
            assert np.linalg.norm(x1[k] - x0[k]) <= 1e-6 * u, (sd, k)
        tot[0] += [sum(s["newton_iters"] for s in s0), sum(s["pcg_iters"] for s in s0)]
        tot[1] += [sum(s["newton_iters"] for s in s1), sum(s["pcg_iters"] for s in s1)]
        taken += sum(s["warm_start_used"] for s in s1)
    say("held-out steps", 2 * steps, "learned start taken", taken, "| newton without/with", tot[0][0], tot[1][0],
        "| pcg without/with", tot[0][1], tot[1][1], "| pcg ratio", tot[1][1] / max(1, tot[0][1]))
