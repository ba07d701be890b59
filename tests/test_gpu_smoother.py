"""GPU tests of the aggregate block-Jacobi smoother (ms_solver_params.smoother
= 1): exact where one aggregate holds the whole system, Newton steps that
land on the oracle's minimiser, fewer PCG iterations than the 3x3 vertex
blocks on the stiff-inclusion block, and the rejected combinations."""
import numpy as np
import pytest

import scenes
from oracle import fem, newton
from tests.gpu_util import device, e_rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def test_single_aggregate_is_exact(dev):
    """The 2 x 2 x 2-vertex cube is one aggregate: its block is the whole
    Hessian (pinned DOFs eliminated), so the preconditioner is H^-1 and each
    FP64 PCG solve reaches a relative residual of 1e-8 in one iteration,
    where the 3x3 blocks need more."""
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(1, seed=0)
    s["v0"] = np.random.default_rng(3).standard_normal(s["rest"].shape)
    c = ms.context_from_scene(dev, s)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    xo, _, _ = newton.newton_step(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](1))
    its = {}
    for sm in (0, 1):
        c.ms_set_state(s["x0"], s["v0"])
        st = c.ms_step(s["dt"], preconditioner=ms.PC_BLOCK_JACOBI, smoother=sm, pcg_eta_max=1e-8, pcg_eta_min=1e-8)
        xg, _ = c.ms_get_state()
        err = e_rel(xg, xo, s["x0"])
        say("single aggregate smoother", sm, "newton", st["newton_iters"], "pcg", st["pcg_iters"],
            "max per solve", st["max_pcg_iters"], "e_rel", err)
        assert err <= 1e-6
        its[sm] = st["max_pcg_iters"]
    assert its[1] == 1 and its[0] > 1
    c.close()


@pytest.mark.parametrize("pc_name,prec_name", [("jacobi", "fp64"), ("additive", "fp64"), ("additive", "mixed")])
def test_aggregate_steps_match_oracle(dev, pc_name, prec_name):
    """Three driven steps of the stiff-inclusion block at 8^3 (9 vertices per
    axis: ragged aggregates on one side, pinned faces inside aggregates)."""
    from paper_2508_13386_amd import ms
    pc = {"jacobi": ms.PC_BLOCK_JACOBI, "additive": ms.PC_TWO_LEVEL_ADDITIVE}[pc_name]
    prec = {"fp64": ms.PREC_FP64, "mixed": ms.PREC_MIXED}[prec_name]
    s = scenes.inclusion_block(8, seed=0, steps=3)
    c = ms.context_from_scene(dev, s)
    if pc != ms.PC_BLOCK_JACOBI:
        c.ms_build_basis(n_handles=10, seed=1, rigid_contrast=1e3)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    x, v = s["x0"].copy(), s["v0"].copy()
    for k in range(1, 4):
        xo, vo, _ = newton.newton_step(body, x, v, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](k))
        c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        c.ms_set_state(x, v)
        st = c.ms_step(s["dt"], precision=prec, preconditioner=pc, smoother=1, forcing=1, pcg_eta_max=0.1,
                       pcg_eta_min=1e-3, coarse_move=0.2, endgame_ratio=1e-1)
        xg, _ = c.ms_get_state()
        err = e_rel(xg, xo, x)
        say("aggregate step", k, pc_name, prec_name, "e_rel", err, "pcg", st["pcg_iters"], "newton",
            st["newton_iters"])
        assert err <= 1e-6
        x, v = xo, vo
    c.close()


def test_aggregate_smoother_cuts_iterations(dev):
    """The stiff-inclusion block at 16^3 with the additive two-level
    preconditioner (22 handles): from the same states, the aggregate smoother
    takes fewer PCG iterations than the 3x3 blocks and reaches the same
    steps."""
    from paper_2508_13386_amd import ms
    s = scenes.inclusion_block(16, seed=0, steps=3)
    c = ms.context_from_scene(dev, s)
    c.ms_build_basis(n_handles=22, seed=1, rigid_contrast=1e3)
    x, v = s["x0"].copy(), s["v0"].copy()
    tot = {0: 0, 1: 0}
    for k in range(1, 4):
        c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        res = {}
        for sm in (0, 1):
            c.ms_set_state(x, v)
            st = c.ms_step(s["dt"], precision=ms.PREC_FP64, preconditioner=ms.PC_TWO_LEVEL_ADDITIVE, smoother=sm,
                           forcing=1, pcg_eta_max=0.1, pcg_eta_min=1e-3, coarse_move=0.2)
            res[sm] = c.ms_get_state()
            tot[sm] += st["pcg_iters"]
            say("step", k, "smoother", sm, "pcg", st["pcg_iters"], "newton", st["newton_iters"])
        assert e_rel(res[1][0], res[0][0], x) <= 1e-6
        x, v = res[0]
    say("pcg iterations 3x3 blocks", tot[0], "aggregates", tot[1], "ratio", tot[1] / tot[0])
    assert tot[1] < tot[0]
    c.close()


def test_aggregate_smoother_rejections(dev):
    from paper_2508_13386_amd import ms
    s = scenes.inclusion_block(4, seed=0, steps=1)
    c = ms.context_from_scene(dev, s)
    c.ms_build_basis(n_handles=4, seed=1)
    x0, _ = c.ms_get_state()
    for kw in (dict(smoother=2), dict(smoother=1, preconditioner=ms.PC_TWO_LEVEL),
               dict(smoother=1, preconditioner=ms.PC_TWO_LEVEL_VCYCLE), dict(smoother=1, mode=ms.MODE_PAPER)):
        with pytest.raises(ms.MSError) as e:
            c.ms_step(s["dt"], **kw)
        assert e.value.code == ms.MS_E_ARG
        assert np.array_equal(c.ms_get_state()[0], x0)
    c2 = ms.context_from_scene(dev, s)
    with pytest.raises(ms.MSError) as e:
        ms.ms_batch_step([c, c2], s["dt"], smoother=1)
    assert e.value.code == ms.MS_E_ARG
    c2.close()
    c.close()
