"""GPU parity of the plain FP64 path against the CPU oracle.

Element terms (energy, gradient, PSD-projected Hessian) at a deformed state,
sliced-BSR3 SpMV, and whole implicit Euler steps at relative displacement
error <= 1e-6 (the gate stated for the plain path)."""
import numpy as np
import pytest

import scenes
from oracle import fem, linops, newton
from tests.gpu_util import device, e_rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _ctx(dev, s, step=1):
    from paper_2508_13386_amd import ms
    return ms.context_from_scene(dev, s, step)


def test_eval_matches_oracle(dev):
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(4, seed=1)
    rng = np.random.default_rng(0)
    s["v0"] = rng.standard_normal(s["rest"].shape)
    c = _ctx(dev, s)
    x = s["rest"] + 0.05 * rng.standard_normal(s["rest"].shape) / 4
    say("eval plain_cube_4")
    e4, g, Hb = c.ms_eval(x, s["dt"], ms.PREC_FP64)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    prob = fem.StepProblem(body, s["x0"], s["v0"], s["dt"], s["gravity"])
    parts = prob.energy_parts(x)
    ref = np.array([parts["K"], parts["Psi"], parts["G"], parts["B"]])
    assert np.allclose(e4, ref, rtol=1e-12, atol=1e-15 * np.abs(ref).sum())
    gref = prob.gradient(x)
    assert np.linalg.norm(g - gref) <= 1e-12 * np.linalg.norm(gref)
    rp, col = c.ms_get_pattern()
    H = linops.bsr_matrix(rp, col, Hb, len(x)).toarray()
    Href = prob.hessian(x).toarray()
    assert np.abs(H - Href).max() <= 1e-11 * np.abs(Href).max()
    # FP32 Hessian within single-precision rounding
    _, _, Hb32 = c.ms_eval(x, s["dt"], ms.PREC_MIXED)
    H32 = linops.bsr_matrix(rp, col, Hb32, len(x)).toarray()
    assert np.abs(H32 - Href).max() <= 2e-6 * np.abs(Href).max()
    c.close()


def test_eval_with_barrier(dev):
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(3, seed=2)
    s["dirichlet"] = np.zeros(0, np.int32)
    s["halfspace"] = dict(normal=np.array([0.0, 0.0, 1.0]), offset=-0.002, dhat=5e-3, kappa=3e4)
    c = _ctx(dev, s)
    rng = np.random.default_rng(1)
    x = s["rest"] + 0.001 * rng.standard_normal(s["rest"].shape)
    x[:, 2] = np.maximum(x[:, 2], -0.0015)
    say("eval barrier")
    e4, g, Hb = c.ms_eval(x, s["dt"])
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    prob = fem.StepProblem(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["halfspace"])
    assert e4[3] > 0
    assert e4[3] == pytest.approx(prob.energy_parts(x)["B"], rel=1e-12)
    gref = prob.gradient(x)
    assert np.linalg.norm(g - gref) <= 1e-12 * np.linalg.norm(gref)
    rp, col = c.ms_get_pattern()
    H = linops.bsr_matrix(rp, col, Hb, len(x)).toarray()
    Href = prob.hessian(x).toarray()
    assert np.abs(H - Href).max() <= 1e-11 * np.abs(Href).max()
    c.close()


def test_energy_difference_matches_oracle(dev):
    """E(x + alpha d) - E(x) by parts (the line-search quantity) equals the
    difference of the oracle's energies where no cancellation hides it, and
    tends to alpha g.d for small alpha (first-order term)."""
    s = scenes.inclusion_block(6, seed=1, steps=1)
    s["halfspace"] = dict(normal=np.array([0.0, 0.0, 1.0]), offset=-0.002, dhat=5e-3, kappa=3e4)
    rng = np.random.default_rng(4)
    s["v0"] = 0.1 * rng.standard_normal(s["rest"].shape)
    c = _ctx(dev, s)
    x = s["rest"] + 0.004 * rng.standard_normal(s["rest"].shape)
    x[:, 2] = np.maximum(x[:, 2], -0.0015)
    d = 0.002 * rng.standard_normal(s["rest"].shape)
    d[:, 2] = np.abs(d[:, 2])  # away from the plane: barrier stays finite
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    prob = fem.StepProblem(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["halfspace"])
    say("energy difference inclusion_block_6")
    alpha = 0.7
    got = c.ms_energy_difference(x, d, alpha, s["dt"])
    p0, p1 = prob.energy_parts(x), prob.energy_parts(x + alpha * d)
    for k, key in enumerate(("K", "Psi", "G", "B")):
        ref = p1[key] - p0[key]
        assert abs(got[k] - ref) <= 1e-9 * (abs(p0[key]) + abs(p1[key])) + 1e-300, key
    assert got[3] != 0.0  # the barrier term is exercised
    assert got[4] >= abs(got[:4]).max()
    # first order: dE / alpha -> g.d
    gd = float((prob.gradient(x) * d).sum())
    a = 1e-7
    small = c.ms_energy_difference(x, d, a, s["dt"])
    assert abs(small[:4].sum() / a - gd) <= 1e-5 * abs(gd)
    c.close()


@pytest.mark.parametrize("dtype,tol", [(0, 1e-13), (1, 1e-5)])
def test_spmv_matches_oracle(dev, dtype, tol):
    import torch
    from paper_2508_13386_amd import ms
    for N, perm in ((5, False), (7, True)):
        rp, col, vals = scenes.spd_bsr_pattern(N, seed=3, permute=perm)
        n = len(rp) - 1
        say("spmv", N, perm, dtype)
        A = ms.Matrix(dev, rp, col, vals, dtype)
        td = torch.float64 if dtype == 0 else torch.float32
        x = np.random.default_rng(4).standard_normal((n, 3))
        xd = torch.tensor(x, dtype=td, device="cuda")
        yd = torch.zeros((n, 3), dtype=td, device="cuda")
        with torch.cuda.stream(dev.stream):
            A.spmv(xd.data_ptr(), yd.data_ptr())
        dev.stream.synchronize()
        y = yd.double().cpu().numpy()
        ref = linops.bsr_matvec(rp, col, vals, x)
        assert np.abs(y - ref).max() <= tol * np.abs(ref).max()
        A.close()


def _run(dev, s, steps, **kw):
    from paper_2508_13386_amd import ms
    c = _ctx(dev, s)
    out = []
    for k in range(1, steps + 1):
        if len(s["dirichlet"]):
            c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        st = c.ms_step(s["dt"], **kw)
        out.append((c.ms_get_state(), st))
    c.close()
    return out


def _oracle_steps(s, steps):
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    x, v = s["x0"].copy(), s["v0"].copy()
    res = []
    for k in range(1, steps + 1):
        xn, vn, _ = newton.newton_step(body, x, v, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](k),
                                       s["halfspace"])
        res.append((x, xn, vn))
        x, v = xn, vn
    return res


def test_plain_cube_step_parity(dev):
    s = scenes.plain_cube(8, seed=0)
    say("plain_cube_8 step")
    (xg, vg), st = _run(dev, s, 1)[0]
    say("stats", st)
    xt, xo, vo = _oracle_steps(s, 1)[0]
    err = e_rel(xg, xo, xt)
    say("e_rel", err)
    assert err <= 1e-6
    assert np.abs(vg - vo).max() <= 1e-6 * np.abs(vo).max() + 1e-12


@pytest.mark.parametrize("projection", [0, 1])
def test_inclusion_block_steps_from_identical_states(dev, projection):
    """Heterogeneous block (E contrast 1e5, nu = 0.49) at 8^3: every step
    starts from the oracle's previous state, so each step is compared from
    identical states; with the eigenvalue clamp and with absolute values in
    the projected Hessians (the minimiser is the same)."""
    from paper_2508_13386_amd import ms
    s = scenes.inclusion_block(8, seed=0, steps=3)
    ref = _oracle_steps(s, 3)
    c = _ctx(dev, s)
    for k, (xt, xo, vo) in enumerate(ref, start=1):
        c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        vt = s["v0"] if k == 1 else ref[k - 2][2]
        c.ms_set_state(xt, vt)
        say("inclusion_block_8 step", k, "projection", projection)
        st = c.ms_step(s["dt"], projection=projection)
        xg, _ = c.ms_get_state()
        err = e_rel(xg, xo, xt)
        say("step", k, "e_rel", err, st)
        assert err <= 1e-6
    c.close()


def test_step_is_deterministic(dev):
    s = scenes.plain_cube(6, seed=3)
    a = _run(dev, s, 2)
    b = _run(dev, s, 2)
    for (sa, _), (sb, _) in zip(a, b):
        assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])


def test_failed_step_leaves_state_unchanged(dev):
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(4, seed=1)
    c = _ctx(dev, s)
    x0, v0 = c.ms_get_state()
    with pytest.raises(ms.MSError) as ei:
        c.ms_step(s["dt"], max_newton=1)
    assert ei.value.code == ms.MS_E_NOCONV
    x1, v1 = c.ms_get_state()
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
    c.close()


def test_block_jacobi_preconditioner_is_spd(dev):
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(4, seed=1)
    c = _ctx(dev, s)
    c.ms_eval(s["x0"], s["dt"])
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((2, len(s["rest"]), 3))
    za = c.ms_apply_preconditioner(ms.PC_BLOCK_JACOBI, a)
    zb = c.ms_apply_preconditioner(ms.PC_BLOCK_JACOBI, b)
    free = np.ones(len(a), bool)
    free[s["dirichlet"]] = False
    assert abs((za * b)[free].sum() - (zb * a)[free].sum()) <= 1e-12 * np.abs(za * b).sum()
    assert (za * a)[free].sum() > 0
    assert np.abs(za[~free]).max() == 0.0
    c.close()


@pytest.mark.parametrize("scene", ["plain_cube", "sliding_cube"])
def test_bdf2_trajectory_matches_oracle(dev, scene):
    """BDF2 (implicit Euler for the first step, which has no history): the
    GPU trajectory against the oracle's, step by step."""
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(4, seed=3) if scene == "plain_cube" else scenes.sliding_cube(4)
    c = _ctx(dev, s)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    x, v, prev = s["x0"].copy(), s["v0"].copy(), None
    if scene == "plain_cube":
        v = 0.5 * np.random.default_rng(2).standard_normal(x.shape)
        v[s["dirichlet"]] = 0.0
        c.ms_set_state(x, v)
    for k in range(1, 5):
        tgt = s["dbc_targets"](k)
        xo, vo, _ = newton.newton_step(body, x, v, s["dt"], s["gravity"], s["dirichlet"], tgt,
                                       halfspace=s["halfspace"], prev=prev)
        if len(s["dirichlet"]):
            c.ms_set_dirichlet(s["dirichlet"], tgt)
        st = c.ms_step(s["dt"], integrator=1)
        xg, vg = c.ms_get_state()
        err = e_rel(xg, xo, x)
        verr = float(np.linalg.norm(vg - vo) / np.linalg.norm(vo))
        say("bdf2", scene, "step", k, "e_rel", err, "v rel", verr, "newton", st["newton_iters"])
        assert err <= 1e-6 and verr <= 1e-6
        prev = (x, v)
        x, v = xo, vo
    c.close()
