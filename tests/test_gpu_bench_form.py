"""The benchmarked workload at its full size, in the form bench.py times,
against the CPU oracle: the heterogeneous block at 32^3 (35,937 vertices,
196,608 tets, 20 inclusions at 1e10 Pa in 1e5 Pa), mixed precision (FP32
Hessian values, FP64 vectors, gradients and line search), the additive
two-level preconditioner on a 144-handle basis with constant weights on
the inclusions and 2x2x2 vertex aggregates as its block part,
Eisenstat-Walker forcing in [3e-2, 0.1], the exact (unprojected) Hessian
from ||d|| <= 1e-1 ||x - x^t||, coarse rebuilds after a movement of
0.8 ||x - x^t|| and at most 200 Newton iterations.

The oracle's sparse direct solve costs about a minute per Newton iteration
at this size, so it starts from the GPU's result (the minimiser does not
depend on the first iterate): one or two exact Newton corrections land on
its own minimiser, and e_rel = ||x_orc - x_gpu|| / ||x_orc - x^t|| is the
GPU's distance to it.  The step checked is the third of the drive, the
first one inside bench.py's timed region."""
import time

import numpy as np
import pytest

import scenes
from oracle import fem, newton
from tests.gpu_util import device, e_rel, say

pytestmark = pytest.mark.gpu


def test_bench_form_step_at_full_size():
    from paper_2508_13386_amd import ms
    dev = device()
    s = scenes.inclusion_block(32, seed=0, steps=3)
    c = ms.context_from_scene(dev, s)
    t0 = time.time()
    c.ms_build_basis(n_handles=144, oversample=1.0, rigid_contrast=1e3)
    say("basis", c.ms_get_basis()["m"], "handles in", round(time.time() - t0, 1), "s")
    params = ms.solver_defaults(precision=ms.PREC_MIXED, preconditioner=ms.PC_TWO_LEVEL_ADDITIVE, forcing=1,
                                pcg_eta_max=0.1, pcg_eta_min=3e-2, coarse_move=0.8, mixed_endgame_fp64=0, smoother=1,
                                endgame_ratio=1e-1, max_newton=200)
    for k in (1, 2):
        c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        c.ms_step(s["dt"], params)
    x2, v2 = c.ms_get_state()
    c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](3))
    st = c.ms_step(s["dt"], params)
    x3, _ = c.ms_get_state()
    c.close()
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    rec = []
    t0 = time.time()
    xo, _, its = newton.newton_step(body, x2, v2, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](3),
                                    x_start=x3, record=rec)
    err = e_rel(x3, xo, x2)
    say("32^3 bench form step 3: newton", st["newton_iters"], "pcg", st["pcg_iters"], "| oracle from the GPU state:",
        its, "iterations,", round(time.time() - t0, 1), "s, last |d|_inf", rec[-1]["dinf"] if rec else None,
        "| e_rel", err)
    assert err <= 1e-6


def test_fp64_continuation_converges_at_full_size():
    """The bench form on a basis of 144 handles (jump penalty 0.35): one of the
    first five driven steps does not converge in 20 mixed-precision Newton
    iterations and continues in FP64.  The continuation uses the FP64 coarse
    inverse (rounded to FP32 the inverse of this ill-conditioned coarse
    matrix made the step fail); every step converges and the states match
    the same steps solved in FP64 throughout."""
    from paper_2508_13386_amd import ms
    dev = device()
    s = scenes.inclusion_block(32, seed=0, steps=5)
    form = dict(preconditioner=ms.PC_TWO_LEVEL_ADDITIVE, forcing=1, pcg_eta_max=0.1, pcg_eta_min=3e-2,
                coarse_move=0.8, mixed_endgame_fp64=0, smoother=1, endgame_ratio=1e-1, max_newton=200)
    states, basis = {}, {}
    for prec in (ms.PREC_MIXED, ms.PREC_FP64):
        c = ms.context_from_scene(dev, s)
        if not basis:
            c.ms_build_basis(n_handles=144, oversample=1.0, jump_penalty=0.35, rigid_contrast=1e3)
            basis.update(c.ms_get_basis())
        else:
            c.ms_set_basis(basis["origins"], basis["vptr"], basis["vhandle"], basis["vphi"])
        esc = []
        for k in range(1, 6):
            c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
            st = c.ms_step(s["dt"], ms.solver_defaults(precision=prec, **form))
            esc.append(st["precision_escalations"])
            say("prec", prec, "step", k, "newton", st["newton_iters"], "pcg", st["pcg_iters"], "escalations",
                st["precision_escalations"])
        states[prec] = c.ms_get_state()[0]
        c.close()
        if prec == ms.PREC_MIXED:
            assert sum(esc) >= 1
    err = e_rel(states[ms.PREC_MIXED], states[ms.PREC_FP64], s["x0"])
    say("mixed vs FP64 after 5 steps: e_rel", err)
    assert err <= 1e-6
