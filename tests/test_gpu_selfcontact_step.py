"""IPC self-contact inside the GPU Newton step, against the CPU oracle.

Two Kuhn cubes in one mesh (the upper one turned and off-centre, falling
onto the lower one, whose bottom is pinned) meet only through point-triangle
and edge-edge barriers.  Checked: the step energy and gradient at a state
with active pairs (ms_eval), the energy difference along a direction, and
whole steps from identical states against oracle.newton.newton_step with
the same self-contact term (e_rel <= 1e-6; the oracle starts from the GPU's
result, the minimiser does not depend on the first iterate), in FP64 and
mixed precision, with block-Jacobi and the additive two-level
preconditioner; the surfaces stay apart and the contact is active."""
import numpy as np
import pytest
import torch

import scenes
from oracle import fem, newton
from oracle import selfcontact as sco
from tests.gpu_util import device, e_rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _min_distance(x, surf, dhat):
    pairs = sco.active_pairs_filtered(x, surf, dhat)
    d = []
    for kind, lst in (("pt", pairs[0]), ("ee", pairs[1])):
        f = sco.pt_dist2 if kind == "pt" else sco.ee_dist2
        for q in lst:
            d.append(float(f(torch.tensor(x[list(q)].ravel(), dtype=torch.float64))))
    return (np.sqrt(min(d)) if d else np.inf), len(pairs[0]) + len(pairs[1])


def test_eval_energy_gradient_and_difference_match_oracle(dev):
    from paper_2508_13386_amd import ms
    s = scenes.stacked_cubes(N=2)
    c = ms.context_from_scene(dev, s)
    x = s["x0"].copy()
    x[s["n_lower"]:, 2] -= 0.5e-3  # gap 0.5 mm, inside d_hat = 2 mm
    e4, g, _ = c.ms_eval(x, s["dt"], hess=False)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    prob = fem.StepProblem(body, s["x0"], s["v0"], s["dt"], s["gravity"], selfcontact=s["selfcontact"])
    parts = prob.energy_parts(x)
    say("contact energy (GPU part 3, oracle C)", e4[3], parts["C"])
    assert parts["C"] > 0.0
    assert abs(e4[3] - parts["C"]) <= 1e-12 * abs(parts["C"])
    go = prob.gradient(x)
    free = np.ones(len(x), bool)
    free[s["dirichlet"]] = False
    err = np.abs(g - go)[free].max() / np.abs(go[free]).max()
    say("gradient rel err", err)
    assert err <= 1e-10
    # energy difference along a downward move of the upper cube
    d = np.zeros_like(x)
    d[s["n_lower"]:, 2] = -0.2e-3
    out = c.ms_energy_difference(x, d, 1.0, s["dt"])
    ref = prob.energy(x + d) - prob.energy(x)
    say("dE GPU", out[:4].sum(), "oracle", ref)
    assert abs(out[:4].sum() - ref) <= 1e-9 * abs(ref) + 1e-14 * out[4]
    c.close()


@pytest.mark.parametrize("prec_name,pc_name,N", [("fp64", "jacobi", 2), ("mixed", "jacobi", 2),
                                                 ("mixed", "additive", 3), ("fp64", "vcycle", 2)])
def test_self_contact_steps_match_oracle(dev, prec_name, pc_name, N):
    from paper_2508_13386_amd import ms
    s = scenes.stacked_cubes(N=N)
    c = ms.context_from_scene(dev, s)
    prec = ms.PREC_MIXED if prec_name == "mixed" else ms.PREC_FP64
    pc = {"jacobi": ms.PC_BLOCK_JACOBI, "additive": ms.PC_TWO_LEVEL_ADDITIVE, "vcycle": ms.PC_TWO_LEVEL_VCYCLE}[pc_name]
    if pc != ms.PC_BLOCK_JACOBI:
        c.ms_build_basis(n_handles=4, seed=1)
    params = ms.solver_defaults(precision=prec, preconditioner=pc, forcing=1, pcg_eta_max=0.1, pcg_eta_min=1e-4)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    surf = sco.surface(s["tets"])
    dhat = s["selfcontact"]["dhat"]
    x, v = c.ms_get_state()
    active = 0
    for k in range(1, 4):
        st = c.ms_step(s["dt"], params)
        x1, v1 = c.ms_get_state()
        xo, _, its = newton.newton_step(body, x, v, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](k),
                                        selfcontact=s["selfcontact"], x_start=x1)
        err = e_rel(x1, xo, x)
        dmin, npairs = _min_distance(x1, surf, dhat)
        active = max(active, npairs)
        gap = x1[s["n_lower"]:, 2].min() - x1[:s["n_lower"], 2].max()
        say(prec_name, pc_name, "step", k, "newton", st["newton_iters"], "pcg", st["pcg_iters"], "min alpha",
            st["min_alpha"], "| oracle its", its, "e_rel", err, "| pairs", npairs, "min d", dmin, "gap", gap)
        assert err <= 1e-6
        assert dmin > 0.0
        x, v = x1, v1
    assert active > 0
    c.close()


def test_free_collision_conserves_momentum(dev):
    from paper_2508_13386_amd import ms
    s = scenes.stacked_cubes(N=2, free=True, speed=0.3)
    c = ms.context_from_scene(dev, s)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    p0 = (body.mass[:, None] * s["v0"]).sum(axis=0)
    scale = np.abs(body.mass[:, None] * s["v0"]).sum()
    for k in range(3):
        c.ms_step(s["dt"], precision=ms.PREC_FP64)
    x, v = c.ms_get_state()
    p = (body.mass[:, None] * v).sum(axis=0)
    say("momentum drift", np.abs(p - p0).max() / scale, "approach speed", v[s["n_lower"]:, 2].mean() -
        v[:s["n_lower"], 2].mean())
    assert np.abs(p - p0).max() <= 1e-7 * scale
    c.close()


def test_self_contact_rejections(dev):
    from paper_2508_13386_amd import ms
    s = scenes.stacked_cubes(N=2)
    c = ms.context_from_scene(dev, s)
    with pytest.raises(ms.MSError) as e:
        c.ms_step(s["dt"], mode=ms.MODE_PAPER)
    assert e.value.code == ms.MS_E_ARG
    c.ms_build_basis(n_handles=4, seed=1)
    with pytest.raises(ms.MSError) as e:
        c.ms_step(s["dt"], preconditioner=ms.PC_TWO_LEVEL)
    assert e.value.code == ms.MS_E_ARG
    with pytest.raises(ms.MSError) as e:  # after the material
        c.ms_set_self_contact(1e-3, 1.0)
    assert e.value.code == ms.MS_E_ORDER
    c2 = ms.context_from_scene(dev, scenes.stacked_cubes(N=2))
    with pytest.raises(ms.MSError) as e:
        ms.ms_batch_step([c, c2], s["dt"])
    assert e.value.code == ms.MS_E_ARG
    c.close()
    c2.close()
    c3 = ms.Context(dev)
    c3.ms_upload_mesh(s["rest"], s["tets"])
    for bad in ((0.0, 1.0, 16), (1e-3, 0.0, 16), (1e-3, 1.0, 0), (1e-3, 1.0, 65)):
        with pytest.raises(ms.MSError) as e:
            c3.ms_set_self_contact(*bad)
        assert e.value.code == ms.MS_E_ARG
    c3.close()


def test_self_contact_with_half_space_matches_oracle(dev):
    """Both contact models at once: the lower cube is not pinned but rests on
    a rigid half-space half a millimetre below it (inside d_hat) while the
    upper one falls onto it; two steps against the oracle with the same
    half-space barrier and self-contact term."""
    from paper_2508_13386_amd import ms
    s = scenes.stacked_cubes(N=2)
    s["dirichlet"] = np.zeros(0, np.int32)
    s["dbc_targets"] = lambda k: np.zeros((0, 3))
    s["halfspace"] = dict(normal=np.array([0.0, 0.0, 1.0]), offset=-0.5e-3, dhat=2e-3,
                          kappa=s["selfcontact"]["kappa"])
    c = ms.context_from_scene(dev, s)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    x, v = c.ms_get_state()
    for k in range(1, 3):
        st = c.ms_step(s["dt"], precision=ms.PREC_MIXED, forcing=1, pcg_eta_max=0.1, pcg_eta_min=1e-4)
        x1, v1 = c.ms_get_state()
        xo, _, its = newton.newton_step(body, x, v, s["dt"], s["gravity"], halfspace=s["halfspace"],
                                        selfcontact=s["selfcontact"], x_start=x1)
        err = e_rel(x1, xo, x)
        say("half-space + self-contact step", k, "newton", st["newton_iters"], "oracle its", its, "e_rel", err,
            "lowest z", float(x1[:, 2].min()))
        assert err <= 1e-6
        assert x1[:, 2].min() > -0.5e-3
        x, v = x1, v1
    c.close()
