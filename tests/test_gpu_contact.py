"""GPU parity of timesteps with IPC half-space contact (Sec. 3.1 barrier,
Sec. 3.7 filtered line search) against the CPU oracle, and the momentum
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
