"""Pins of the oracle's Newton timestep: closed-form free fall, momentum
conservation, zero-force rest state, energy decrease, dense brute force,
contact filter, and the textbook linear-elastic limit."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import scenes
from oracle import fem, newton


def _body(N=2, E=1e6, nu=0.45, seed=0):
    rest, tets, _, _ = scenes.kuhn_cube(N)
    T = len(tets)
    return fem.Body(rest, tets, np.full(T, E), np.full(T, nu), np.full(T, 1000.0)), rest


def test_rest_state_exits_immediately():
    body, rest = _body()
    x, v, its = newton.newton_step(body, rest, np.zeros_like(rest), 0.01, np.zeros(3))
    assert np.array_equal(x, rest) and its == 1
    assert np.abs(v).max() == 0.0


def test_free_fall_closed_form():
    body, rest = _body()
    g = np.array([0.0, 0.0, -9.81])
    h = 1.0 / 60.0
    v0 = np.tile([0.3, -0.1, 0.2], (len(rest), 1))
    x, v, _ = newton.newton_step(body, rest, v0, h, g)
    assert np.allclose(x, rest + h * v0 + h * h * g, rtol=0, atol=1e-13)
    assert np.allclose(v, v0 + h * g, rtol=0, atol=1e-11)


def test_momentum_conserved_without_external_forces():
    body, rest = _body(N=2, E=1e5)
    rng = np.random.default_rng(3)
    x0 = rest + 0.02 * rng.standard_normal(rest.shape)
    v0 = rng.standard_normal(rest.shape)
    x, v, _ = newton.newton_step(body, x0, v0, 0.01, np.zeros(3))
    p0 = (body.mass[:, None] * v0).sum(axis=0)
    p1 = (body.mass[:, None] * v).sum(axis=0)
    assert np.allclose(p0, p1, rtol=0, atol=1e-10 * np.abs(body.mass[:, None] * v0).sum())
    # angular momentum of implicit Euler changes; linear momentum must not


def test_energy_decreases_every_iteration():
    s = scenes.inclusion_block(6, seed=1, steps=1)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    rec = []
    newton.newton_step(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](1),
                       record=rec)
    E = [r["E"] for r in rec]
    assert len(E) >= 3
    scale = abs(E[0])
    for a, b in zip(E, E[1:]):
        assert b <= a + 1e-12 * scale


@pytest.mark.parametrize("N", [1, 2])
def test_dense_equals_sparse(N):
    s = scenes.plain_cube(N, seed=2)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    args = (body, s["x0"], s["v0"] + 0.5, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](1))
    xs, _, _ = newton.newton_step(*args)
    xd, _, _ = newton.newton_step(*args, dense=True)
    assert np.allclose(xs, xd, rtol=0, atol=1e-12)


def test_solution_is_stationary_and_matches_brute_force_minimiser():
    """The converged x zeroes the free gradient, and a generic minimiser
    (scipy L-BFGS on the same energy) lands on the same point."""
    from scipy.optimize import minimize
    s = scenes.plain_cube(1, seed=5)
    body = fem.Body(s["rest"], s["tets"], s["E"] * 0 + 1e4, s["nu"], s["rho"])
    v0 = np.zeros_like(s["rest"])
    v0[:, 0] = 1.0
    x, _, _ = newton.newton_step(body, s["x0"], v0, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](1))
    prob = fem.StepProblem(body, s["x0"], v0, s["dt"], s["gravity"])
    free = np.setdiff1d(np.arange(len(x)), s["dirichlet"])
    g = prob.gradient(x)
    assert np.abs(g[free]).max() < 1e-10
    x0 = s["x0"].copy()

    def f(z):
        y = x0.copy()
        y[free] = z.reshape(-1, 3)
        return prob.energy(y), prob.gradient(y)[free].ravel()

    r = minimize(f, x0[free].ravel(), jac=True, method="L-BFGS-B", options=dict(gtol=1e-14, ftol=1e-16, maxiter=5000))
    assert np.allclose(r.x.reshape(-1, 3), x[free], rtol=0, atol=1e-7)


def test_linear_elastic_limit():
    """Tiny load: Newton's displacement equals the textbook linear-elastic
    implicit-Euler solve (M + h^2 K) u = h^2 M g to O(load)."""
    s = scenes.plain_cube(3, seed=0)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    gsmall = s["gravity"] * 1e-4
    h = s["dt"]
    x, _, _ = newton.newton_step(body, s["x0"], s["v0"], h, gsmall, s["dirichlet"], s["dbc_targets"](1))
    u_nl = (x - s["x0"]).ravel()
    # textbook stiffness V B^T D B in Voigt notation, written independently of the SNH code
    rest, tets = s["rest"], s["tets"]
    n3 = 3 * len(rest)
    rows, cols, vals = [], [], []
    for t in range(len(tets)):
        X = rest[tets[t]]
        A = np.hstack([np.ones((4, 1)), X])
        grads = np.linalg.inv(A)[1:].T
        V = abs(np.linalg.det(A)) / 6
        Bm = np.zeros((6, 12))
        for a in range(4):
            bx, by, bz = grads[a]
            Bm[:, 3 * a:3 * a + 3] = [[bx, 0, 0], [0, by, 0], [0, 0, bz], [by, bx, 0], [0, bz, by], [bz, 0, bx]]
        e, nu = s["E"][t], s["nu"][t]
        c = e / ((1 + nu) * (1 - 2 * nu))
        D = c * np.diag([1 - nu] * 3 + [(1 - 2 * nu) / 2] * 3)
        D[:3, :3] += c * nu * (1 - np.eye(3))
        K = V * Bm.T @ D @ Bm
        dof = (3 * tets[t][:, None] + np.arange(3)).ravel()
        rows.append(np.repeat(dof, 12))
        cols.append(np.tile(dof, 12))
        vals.append(K.ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n3, n3)).tocsr()
    m = np.zeros(len(rest))
    vol = np.array([abs(np.linalg.det(np.hstack([np.ones((4, 1)), rest[t]]))) / 6 for t in tets])
    np.add.at(m, tets.ravel(), np.repeat(s["rho"] * vol / 4, 4))
    A = sp.diags(np.repeat(m, 3)) + h * h * K
    f = h * h * np.repeat(m, 3) * np.tile(gsmall, len(rest))
    free = np.ones(n3, bool)
    free[(3 * s["dirichlet"][:, None] + np.arange(3)).ravel()] = False
    u_lin = np.zeros(n3)
    u_lin[free] = spla.spsolve(A[free][:, free].tocsc(), f[free])
    rel = np.linalg.norm(u_nl - u_lin) / np.linalg.norm(u_lin)
    assert rel < 1e-3


def test_contact_filter_keeps_vertices_above_plane():
    body, rest = _body(N=2, E=1e6)
    x0 = rest + np.array([0.0, 0.0, 0.004])
    v0 = np.zeros_like(rest)
    v0[:, 2] = -3.0
    hs = dict(normal=np.array([0.0, 0.0, 1.0]), offset=0.0, dhat=5e-3, kappa=1e4)
    x = x0
    v = v0
    for _ in range(5):
        x, v, _ = newton.newton_step(body, x, v, 0.01, np.array([0.0, 0.0, -9.81]), halfspace=hs)
        assert x[:, 2].min() > 0.0
    prob = fem.StepProblem(body, x, v, 0.01, np.array([0.0, 0.0, -9.81]), hs)
    assert fem.barrier(x[:, 2], 5e-3).sum() > 0  # in contact
    assert newton.ccd_bound(x, np.tile([0.0, 0.0, -1.0], (len(x), 1)), hs) == pytest.approx(0.9 * x[:, 2].min())


def test_bdf2_free_fall_is_exact():
    """BDF2 is exact on trajectories quadratic in time: an unconstrained,
    undeformed body in free fall, started with the exact history, follows
    x(t) = x0 + v0 t + g t^2 / 2 to round-off (this also fixes the weight
    4/9 on the h^2 terms)."""
    rest, tets, _, _ = scenes.kuhn_cube(2)
    T = len(tets)
    body = fem.Body(rest, tets, np.full(T, 1e6), np.full(T, 0.3), np.full(T, 1000.0))
    g = np.array([0.0, 0.0, -9.81])
    v0 = np.array([0.3, -0.2, 1.0])
    h = 0.01
    X = lambda t: rest + v0 * t + 0.5 * g * t * t
    V = lambda t: np.tile(v0 + g * t, (len(rest), 1))
    for k in range(1, 4):
        x, v, _ = newton.newton_step(body, X(k * h), V(k * h), h, g, prev=(X((k - 1) * h), V((k - 1) * h)))
        assert np.abs(x - X((k + 1) * h)).max() <= 1e-12
        assert np.abs(v - V((k + 1) * h)).max() <= 1e-9


def test_backtracking_phase_does_not_stop_the_newton_iteration():
    """A cube squashed to a fifth of its height springs back: the first Newton
    steps backtrack and their sizes are not monotone (a stagnation rule
    applied there stopped after six iterations with a 1 m step left).  The
    iteration must still end at a minimiser: the last full step is below
    1e-12 of the bounding box and the free gradient has fallen by many
    orders."""
    s = scenes.plain_cube(6, seed=0)
    x0 = s["x0"].copy()
    x0[:, 2] *= 0.2
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    rec = []
    x, _, _ = newton.newton_step(body, x0, s["v0"], s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](1),
                                 record=rec)
    assert any(r["alpha"] < 1.0 for r in rec)
    L = float(np.linalg.norm(s["rest"].max(axis=0) - s["rest"].min(axis=0)))
    assert rec[-1]["alpha"] == 1.0 and rec[-1]["dinf"] <= 1e-12 * L
    prob = fem.StepProblem(body, x0, s["v0"], s["dt"], s["gravity"])
    free = np.ones(len(x0), bool)
    free[s["dirichlet"]] = False
    g0 = np.abs(prob.gradient(x0)[free]).max()
    assert np.abs(prob.gradient(x)[free]).max() <= 1e-9 * g0
