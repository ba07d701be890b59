"""Pins of the oracle's incremental potential against things other than itself:
finite differences, the rest state, rigid motions, closed forms of the barrier
and the textbook isotropic linear-elastic stiffness."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenes
from oracle import fem


def _tiny(seed=0, N=2, perturb=0.08, hs=True):
    rest, tets, _, _ = scenes.kuhn_cube(N)
    rng = np.random.default_rng(seed)
    T = len(tets)
    E = np.exp(rng.uniform(np.log(1e5), np.log(1e7), T))
    body = fem.Body(rest, tets, E, np.full(T, 0.4), np.full(T, 1000.0))
    x = rest + perturb * rng.standard_normal(rest.shape) / N
    v = rng.standard_normal(rest.shape)
    halfspace = None
    if hs:
        # plane just below the lowest vertices so that some are inside dhat
        zmin = x[:, 2].min()
        halfspace = dict(normal=np.array([0.0, 0.0, 1.0]), offset=zmin - 2e-3, dhat=1e-2, kappa=1e4)
    prob = fem.StepProblem(body, rest, v, 1.0 / 60.0, np.array([0.0, 0.0, -9.81]), halfspace)
    return prob, x


def test_gradient_matches_central_differences():
    prob, x = _tiny()
    g = prob.gradient(x).ravel()
    eps = 1e-7
    fd = np.zeros_like(g)
    for k in range(len(g)):
        e = np.zeros(len(g))
        e[k] = eps
        fd[k] = (prob.energy(x + e.reshape(x.shape)) - prob.energy(x - e.reshape(x.shape))) / (2 * eps)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)


def test_hessian_matches_central_differences():
    prob, x = _tiny(seed=1)
    H = prob.hessian(x, project=False).toarray()
    eps = 1e-6
    n3 = H.shape[0]
    fd = np.zeros_like(H)
    for k in range(n3):
        e = np.zeros(n3)
        e[k] = eps
        fd[:, k] = (prob.gradient(x + e.reshape(x.shape)) - prob.gradient(x - e.reshape(x.shape))).ravel() / (2 * eps)
    assert np.linalg.norm(fd - H) <= 1e-5 * np.linalg.norm(H)
    assert np.allclose(H, H.T, rtol=0, atol=1e-9 * np.abs(H).max())


def test_rest_state_is_stress_free():
    mu, lam = np.array([3.0]), np.array([11.0])
    F = np.eye(3)[None]
    assert abs(fem.snh_psi(F, mu, lam)[0]) < 1e-15
    assert np.abs(fem.snh_P(F, mu, lam)).max() < 1e-15
    w = np.sort(np.linalg.eigvalsh(fem.snh_dPdF(F, mu, lam)[0]))
    # derived: 3 lam' - mu (x1, volumetric), 2 mu (x5, deviatoric), 0 (x3, rotations)
    ref = np.sort(np.array([3 * 11.0 - 3.0] + [6.0] * 5 + [0.0] * 3))
    assert np.allclose(w, ref, atol=1e-12)
    # the projection is a no-op at rest
    C = fem.snh_dPdF(F, mu, lam)
    assert np.allclose(fem.project_psd(C), C, atol=1e-12)


def test_rigid_motion_invariance():
    rest, tets, _, _ = scenes.kuhn_cube(2)
    T = len(tets)
    body = fem.Body(rest, tets, np.full(T, 1e6), np.full(T, 0.45), np.full(T, 1000.0))
    R = Rotation.random(random_state=4).as_matrix()
    x = rest @ R.T + np.array([0.3, -2.0, 5.0])
    F = body.deformation_gradient(x)
    assert np.abs(fem.snh_psi(F, body.mu, body.lam)).max() < 1e-9
    prob = fem.StepProblem(body, x, np.zeros_like(x), 0.01, np.zeros(3))
    g = prob.gradient(x)  # inertia term is zero at x = x~
    assert np.abs(g).max() < 1e-9 * 1e6 * 1e-4
    # 6-dimensional null space of the unpinned elastic Hessian at rest
    He = prob.hessian(rest, project=False).toarray() - np.diag(np.repeat(body.mass, 3))
    w = np.linalg.eigvalsh(He)
    assert (np.abs(w) < 1e-8 * np.abs(w).max()).sum() == 6


def test_small_strain_limit_is_textbook_linear_elasticity():
    """lam' = lam + mu: the SNH Hessian at rest equals the isotropic linear
    elastic stiffness V B^T D B written in Voigt notation."""
    rest, tets, _, _ = scenes.kuhn_cube(2)
    rng = np.random.default_rng(2)
    T = len(tets)
    E = rng.uniform(1e5, 1e7, T)
    nu = rng.uniform(0.1, 0.49, T)
    body = fem.Body(rest, tets, E, nu, np.full(T, 1.0))
    prob = fem.StepProblem(body, rest, np.zeros_like(rest), 1.0, np.zeros(3))
    Hsnh = prob.element_hessians(rest, project=False)
    for t in range(T):
        X = rest[tets[t]]
        A = np.hstack([np.ones((4, 1)), X])
        grads = np.linalg.inv(A)[1:].T  # [4,3] gradients of the linear shape functions
        V = abs(np.linalg.det(A)) / 6
        Bm = np.zeros((6, 12))
        for a in range(4):
            bx, by, bz = grads[a]
            Bm[:, 3 * a:3 * a + 3] = [[bx, 0, 0], [0, by, 0], [0, 0, bz], [by, bx, 0], [0, bz, by], [bz, 0, bx]]
        e, n = E[t], nu[t]
        c = e / ((1 + n) * (1 - 2 * n))
        D = c * np.array([[1 - n, n, n, 0, 0, 0], [n, 1 - n, n, 0, 0, 0], [n, n, 1 - n, 0, 0, 0],
                          [0, 0, 0, (1 - 2 * n) / 2, 0, 0], [0, 0, 0, 0, (1 - 2 * n) / 2, 0],
                          [0, 0, 0, 0, 0, (1 - 2 * n) / 2]])
        K = V * Bm.T @ D @ Bm
        assert np.allclose(Hsnh[t], K, rtol=0, atol=1e-10 * np.abs(K).max())


def test_projection_clamps_only_negative_eigenvalues():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    w = np.array([-3.0, -1e-3, 0.0, 0.5, 1, 2, 3, 4, 5])
    A = (Q * w) @ Q.T
    P = fem.project_psd(A[None])[0]
    assert np.allclose(P, (Q * np.maximum(w, 0)) @ Q.T, atol=1e-12)
    # inverted element: projected Hessian is PSD, unprojected is not
    F = np.diag([1.2, 0.9, -0.3])[None]
    C = fem.snh_dPdF(F, np.array([1.0]), np.array([20.0]))
    assert np.linalg.eigvalsh(C[0]).min() < 0
    assert np.linalg.eigvalsh(fem.project_psd(C)[0]).min() > -1e-12


def test_barrier_closed_forms():
    dhat = 1e-3
    d = np.linspace(1e-7, dhat * 0.999999, 2001)
    b, b1, b2 = fem.barrier(d, dhat), fem.barrier_d1(d, dhat), fem.barrier_d2(d, dhat)
    assert (b > 0).all() and (b1 < 0).all() and (b2 > 0).all()
    # C2 at dhat (all three vanish there) and zero beyond
    for f in (fem.barrier, fem.barrier_d1, fem.barrier_d2):
        assert f(np.array([dhat * (1 - 1e-9)]), dhat)[0] == pytest.approx(0.0, abs=1e-6)
        assert f(np.array([1.5 * dhat]), dhat)[0] == 0.0
    # diverges as d -> 0
    assert fem.barrier(np.array([1e-300]), dhat)[0] > 1e-4
    assert np.isinf(fem.barrier(np.array([0.0]), dhat)[0])
    # derivative consistency by central differences
    dd = np.array([1e-5, 1e-4, 5e-4, 9e-4])
    eps = 1e-10
    fd1 = (fem.barrier(dd + eps, dhat) - fem.barrier(dd - eps, dhat)) / (2 * eps)
    fd2 = (fem.barrier_d1(dd + eps, dhat) - fem.barrier_d1(dd - eps, dhat)) / (2 * eps)
    assert np.allclose(fd1, fem.barrier_d1(dd, dhat), rtol=1e-5)
    assert np.allclose(fd2, fem.barrier_d2(dd, dhat), rtol=1e-5)
    # closed form at d = dhat / e: b = (dhat (1 - 1/e))^2
    x = dhat / np.e
    assert fem.barrier(np.array([x]), dhat)[0] == pytest.approx((dhat - x) ** 2, rel=1e-14)


def test_inverted_rest_tet_raises():
    rest, tets, _, _ = scenes.kuhn_cube(1)
    bad = tets.copy()
    bad[0, [2, 3]] = bad[0, [3, 2]]
    with pytest.raises(fem.MeshError):
        fem.Body(rest, bad, np.ones(6), np.full(6, 0.3), np.ones(6))


def test_lumped_mass_total():
    rest, tets, _, _ = scenes.kuhn_cube(3)
    T = len(tets)
    body = fem.Body(rest, tets, np.ones(T), np.full(T, 0.3), np.full(T, 1000.0))
    assert body.mass.sum() == pytest.approx(1000.0, rel=1e-13)


# ---------------------------------------------------------------------------
# friction (lagged IPC form against the half-space)
# ---------------------------------------------------------------------------
def test_friction_magnitude_closed_forms():
    eh = 2e-3
    y = np.array([0.0, 0.3 * eh, eh * (1 - 1e-12), eh, 3 * eh])
    f0, f1, f2 = fem.friction_f0(y, eh), fem.friction_f1(y, eh), fem.friction_f2(y, eh)
    assert f0[0] == pytest.approx(eh / 3.0, rel=1e-15) and f1[0] == 0.0 and f2[0] == pytest.approx(2.0 / eh)
    # C1 at eh (values and slopes from both sides), Coulomb magnitude beyond
    assert f0[2] == pytest.approx(eh, rel=1e-9) and f0[3] == eh and f0[4] == 3 * eh
    assert f1[2] == pytest.approx(1.0, rel=1e-9) and f1[3] == 1.0 and f1[4] == 1.0
    assert abs(f2[2]) <= 1e-6 / eh and f2[4] == 0.0
    # f1 = f0' and f2 = f1' by central differences on both branches
    for yy in (0.2 * eh, 0.7 * eh, 2.5 * eh):
        s = 1e-6 * eh
        assert fem.friction_f1(yy, eh) == pytest.approx(
            (fem.friction_f0(yy + s, eh) - fem.friction_f0(yy - s, eh)) / (2 * s), rel=1e-7, abs=1e-9)
        assert fem.friction_f2(yy, eh) == pytest.approx(
            (fem.friction_f1(yy + s, eh) - fem.friction_f1(yy - s, eh)) / (2 * s), rel=1e-6, abs=1e-6 / eh)


def _tiny_friction(seed=3):
    prob, x = _tiny(seed=seed)
    # plane within dhat of the lowest vertices of x^t, so they carry a lagged normal force
    hs = dict(prob.hs, offset=prob.x_t[:, 2].min() - 3e-3, mu=0.4, eps_v=0.05)
    prob = fem.StepProblem(prob.b, prob.x_t, (prob.xtilde - prob.x_t) / prob.h, prob.h, prob.gravity, hs)
    eh = hs["eps_v"] * prob.h
    # tangential displacements from x^t on both sides of eps_v h
    rng = np.random.default_rng(seed + 1)
    u = rng.standard_normal(x.shape) * np.array([1.0, 1.0, 0.0])
    scale = np.where(np.arange(len(x)) % 2 == 0, 0.4 * eh, 4.0 * eh)
    x = prob.x_t + u / np.linalg.norm(u, axis=1)[:, None] * scale[:, None] + np.array([0, 0, 1e-4])
    assert (prob.fric["mulam"] > 0).sum() >= 2  # some vertices carry a normal force
    return prob, x


def test_friction_gradient_and_hessian_match_central_differences():
    prob, x = _tiny_friction()
    g = prob.gradient(x).ravel()
    H = prob.hessian(x, project=False).toarray()
    eps = 1e-9
    fd_g = np.zeros_like(g)
    fd_H = np.zeros_like(H)
    for k in range(len(g)):
        e = np.zeros(len(g))
        e[k] = eps
        xp, xm = x + e.reshape(x.shape), x - e.reshape(x.shape)
        fd_g[k] = (prob.energy(xp) - prob.energy(xm)) / (2 * eps)
        fd_H[:, k] = (prob.gradient(xp).ravel() - prob.gradient(xm).ravel()) / (2 * eps)
    assert np.linalg.norm(fd_g - g) <= 1e-6 * np.linalg.norm(g)
    assert np.abs(fd_H - H).max() <= 1e-5 * np.abs(H).max()
    # the friction blocks alone are symmetric positive semi-definite
    for blk in prob.friction_blocks(x):
        assert np.allclose(blk, blk.T, atol=1e-12 * np.abs(blk).max() + 1e-300)
        assert np.linalg.eigvalsh(blk).min() >= -1e-9 * max(np.abs(blk).max(), 1e-300)


def test_friction_decelerates_a_sliding_body_by_mu_g_h():
    """Coulomb's law: a stiff cube resting on the plane (normal force = its
    weight) and sliding tangentially loses mu * M * g * h of tangential
    momentum in one implicit step, whatever the barrier's constants."""
    from oracle import newton
    rest, tets, _, _ = scenes.kuhn_cube(2, size=0.1)
    T = len(tets)
    body = fem.Body(rest, tets, np.full(T, 1e9), np.full(T, 0.3), np.full(T, 1000.0))
    g = np.array([0.0, 0.0, -9.81])
    hs = dict(normal=np.array([0.0, 0.0, 1.0]), offset=-5e-4, dhat=1e-3, kappa=1e5)
    # static equilibrium on the plane: one step so long that inertia vanishes
    x_eq, _, _ = newton.newton_step(body, rest, np.zeros_like(rest), 30.0, g, halfspace=hs)
    M = body.mass.sum()
    mu, h, v0 = 0.3, 0.01, np.array([1.0, 0.5, 0.0])
    hsf = dict(hs, mu=mu, eps_v=1e-4)
    v_t = np.tile(v0, (len(rest), 1))
    x1, v1, _ = newton.newton_step(body, x_eq, v_t, h, g, halfspace=hsf)
    dp = (body.mass[:, None] * (v1 - v_t)).sum(axis=0)
    expect = -h * mu * M * 9.81 * v0 / np.linalg.norm(v0)
    assert np.abs(dp[:2] - expect[:2]).max() <= 1e-4 * np.linalg.norm(expect)
