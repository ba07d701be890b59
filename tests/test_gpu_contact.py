"""GPU parity of timesteps with IPC half-space contact (Sec. 3.1 barrier,
Sec. 3.9 filtered line search) against the CPU oracle, and the momentum
balance that every converged contact step satisfies."""
import numpy as np
import pytest

import scenes
from oracle import fem, newton
from tests.gpu_util import device, e_rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_contact_steps_match_oracle(dev, prec_name):
    """A gyroid-masked sphere (res 16: 1,969 vertices, 3,396 tets) hits the
    slab at 5 m/s; each GPU step starts from the oracle's state."""
    from paper_2508_13386_amd import ms
    prec = ms.PREC_MIXED if prec_name == "mixed" else ms.PREC_FP64
    s = scenes.gyroid_sphere(res=16)
    c = ms.context_from_scene(dev, s)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    x, v = s["x0"].copy(), s["v0"].copy()
    dhat = s["halfspace"]["dhat"]
    active = 0
    for k in range(1, 4):
        xo, vo, _ = newton.newton_step(body, x, v, s["dt"], s["gravity"], None, None, halfspace=s["halfspace"])
        c.ms_set_state(x, v)
        st = c.ms_step(s["dt"], precision=prec)
        xg, vg = c.ms_get_state()
        err = e_rel(xg, xo, x)
        active += int((xg[:, 2] < dhat).sum())
        say("contact step", k, prec_name, "e_rel", err, "newton", st["newton_iters"], "pcg", st["pcg_iters"],
            "min z", xg[:, 2].min())
        assert err <= 1e-6
        assert (xg[:, 2] > 0).all()  # the filter keeps every vertex off the slab
        x, v = xo, vo
    assert active > 0  # the barrier was active
    c.close()


def test_contact_momentum_balance(dev):
    """Summed over vertices, the converged step satisfies
    sum m (v^{t+1} - v^t) / h = sum m g - kappa sum b'(d_v) n
    (internal elastic forces cancel), at every step of a bounce."""
    from paper_2508_13386_amd import ms
    s = scenes.gyroid_sphere(res=16)
    c = ms.context_from_scene(dev, s)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    m = body.mass
    hs = s["halfspace"]
    n = np.asarray(hs["normal"])
    weight = m.sum() * np.asarray(s["gravity"])
    x, v = c.ms_get_state()
    worst = 0.0
    for k in range(1, 21):
        st = c.ms_step(s["dt"])
        x1, v1 = c.ms_get_state()
        d = x1 @ n - hs["offset"]
        barrier = -hs["kappa"] * fem.barrier_d1(d, hs["dhat"]).sum() * n
        lhs = (m[:, None] * (v1 - v)).sum(axis=0) / s["dt"]
        rhs = weight + barrier
        scale = np.linalg.norm(weight) + np.linalg.norm(barrier) + np.linalg.norm(lhs)
        err = np.linalg.norm(lhs - rhs) / scale
        worst = max(worst, err)
        say("balance step", k, "err", err, "barrier", barrier[2], "newton", st["newton_iters"])
        assert err <= 1e-6
        x, v = x1, v1
    c.close()


def test_eval_with_friction_matches_oracle(dev):
    """Energy, gradient and Hessian with lagged friction at a state that has
    vertices on both sides of the smoothing length eps_v h."""
    from paper_2508_13386_amd import ms
    from oracle import linops
    s = scenes.sliding_cube(3)
    c = ms.context_from_scene(dev, s)
    rng = np.random.default_rng(4)
    eh = s["halfspace"]["eps_v"] * s["dt"]
    u = rng.standard_normal(s["rest"].shape) * np.array([1.0, 1.0, 0.0])
    scale = np.where(np.arange(len(u)) % 2 == 0, 0.3 * eh, 5.0 * eh)
    x = s["x0"] + u / np.linalg.norm(u, axis=1)[:, None] * scale[:, None]
    say("eval friction")
    e4, g, Hb = c.ms_eval(x, s["dt"])
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    prob = fem.StepProblem(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["halfspace"])
    parts = prob.energy_parts(x)
    assert parts["D"] > 0
    assert e4[3] == pytest.approx(parts["B"] + parts["D"], rel=1e-12)
    gref = prob.gradient(x)
    assert np.linalg.norm(g - gref) <= 1e-12 * np.linalg.norm(gref)
    rp, col = c.ms_get_pattern()
    H = linops.bsr_matrix(rp, col, Hb, len(x)).toarray()
    Href = prob.hessian(x).toarray()
    assert np.abs(H - Href).max() <= 1e-11 * np.abs(Href).max()
    c.close()


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_friction_steps_match_oracle(dev, prec_name):
    """A cube sliding on the slab at 1.1 m/s with mu = 0.5 (lagged friction
    against the half-space); each GPU step starts from the oracle's state and
    the slide decelerates by about mu g h per step."""
    from paper_2508_13386_amd import ms
    prec = ms.PREC_MIXED if prec_name == "mixed" else ms.PREC_FP64
    s = scenes.sliding_cube(6)
    c = ms.context_from_scene(dev, s)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    x, v = s["x0"].copy(), s["v0"].copy()
    mu, h = s["halfspace"]["mu"], s["dt"]
    for k in range(1, 4):
        xo, vo, _ = newton.newton_step(body, x, v, h, s["gravity"], None, None, halfspace=s["halfspace"])
        c.ms_set_state(x, v)
        st = c.ms_step(h, precision=prec)
        xg, vg = c.ms_get_state()
        err = e_rel(xg, xo, x)
        dv = np.linalg.norm((body.mass[:, None] * vg).sum(0)[:2]) - np.linalg.norm((body.mass[:, None] * v).sum(0)[:2])
        say("friction step", k, prec_name, "e_rel", err, "newton", st["newton_iters"], "pcg", st["pcg_iters"],
            "tangential speed change", dv / body.mass.sum(), "mu g h", mu * 9.81 * h)
        assert err <= 1e-6
        assert dv < 0  # friction opposes the slide
        x, v = xo, vo
    c.close()


def test_paper_mode_rejects_friction(dev):
    from paper_2508_13386_amd import ms
    s = scenes.sliding_cube(3)
    c = ms.context_from_scene(dev, s)
    c.ms_build_basis(n_handles=4, seed=0)
    with pytest.raises(ms.MSError) as e:
        c.ms_step(s["dt"], mode=ms.MODE_PAPER)
    assert e.value.code == ms.MS_E_ARG
    c.close()
