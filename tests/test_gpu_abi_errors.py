"""Error contracts of the C ABI on a device: call order, degenerate and
non-finite input, and the transactional timestep (a failed ms_step leaves x,
v and the BDF2 history as they were)."""
import numpy as np
import pytest

import scenes
from oracle import fem, newton
from tests.gpu_util import device, e_rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _code(fn, *a, **kw):
    from paper_2508_13386_amd import ms
    try:
        fn(*a, **kw)
    except ms.MSError as e:
        return e.code
    return ms.MS_OK


def test_call_order(dev):
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(2, seed=0)
    c = ms.Context(dev)
    assert _code(c.ms_upload_material, s["E"], s["nu"], s["rho"]) == ms.MS_E_ORDER
    c.ms_upload_mesh(s["rest"], s["tets"])
    assert _code(c.ms_upload_mesh, s["rest"], s["tets"]) == ms.MS_E_ORDER
    assert _code(c.ms_set_state, s["x0"], s["v0"]) == ms.MS_E_ORDER
    assert _code(c.ms_build_basis, n_handles=2) == ms.MS_E_ORDER
    c.ms_upload_material(s["E"], s["nu"], s["rho"])
    assert _code(c.ms_step, s["dt"]) == ms.MS_E_ORDER
    c.ms_set_state(s["x0"], s["v0"])
    # a two-level step or paper mode without a basis
    assert _code(c.ms_step, s["dt"], preconditioner=ms.PC_TWO_LEVEL_ADDITIVE) == ms.MS_E_ORDER
    assert _code(c.ms_step, s["dt"], mode=ms.MODE_PAPER) == ms.MS_E_ORDER
    c.ms_step(s["dt"])
    c.close()


def test_degenerate_and_nonfinite_input(dev):
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(2, seed=0)
    # an inverted rest tet (two vertices swapped) and a repeated vertex
    for bad in ("inverted", "repeated"):
        tets = s["tets"].copy()
        if bad == "inverted":
            tets[3, [0, 1]] = tets[3, [1, 0]]
        else:
            tets[3, 1] = tets[3, 0]
        c = ms.Context(dev)
        assert _code(c.ms_upload_mesh, s["rest"], tets) == ms.MS_E_MESH, bad
        c.close()
    # non-finite rest positions, material, state and Dirichlet targets
    rest = s["rest"].copy()
    rest[5, 1] = np.nan
    c = ms.Context(dev)
    assert _code(c.ms_upload_mesh, rest, s["tets"]) == ms.MS_E_NONFINITE
    c.close()
    c = ms.Context(dev)
    c.ms_upload_mesh(s["rest"], s["tets"])
    E = s["E"].copy()
    E[0] = np.inf
    assert _code(c.ms_upload_material, E, s["nu"], s["rho"]) == ms.MS_E_NONFINITE
    c.ms_upload_material(s["E"], s["nu"], s["rho"])
    tgt = s["rest"][s["dirichlet"]].copy()
    tgt[0, 2] = np.nan
    assert _code(c.ms_set_dirichlet, s["dirichlet"], tgt) == ms.MS_E_NONFINITE
    v = s["v0"].copy()
    v[2, 0] = np.nan
    assert _code(c.ms_set_state, s["x0"], v) == ms.MS_E_NONFINITE
    # the context is still usable afterwards
    c.ms_set_state(s["x0"], s["v0"])
    assert _code(c.ms_step, -1.0) == ms.MS_E_ARG
    c.ms_step(s["dt"])
    c.close()


def _squashed(N=4):
    s = scenes.plain_cube(N, seed=0)
    x0 = s["x0"].copy()
    x0[:, 2] *= 0.3  # the bottom face stays in place (z = 0)
    return s, x0


def test_line_search_failure_leaves_the_state(dev):
    """The squashed cube's first Newton step needs five halvings (the oracle's
    alpha = 1/32); with no halving allowed the step fails with
    MS_E_LINESEARCH and x, v stay bitwise as set.  The same context then
    steps normally and matches the oracle."""
    from paper_2508_13386_amd import ms
    s, x0 = _squashed()
    c = ms.context_from_scene(dev, s)
    v0 = np.zeros_like(x0)
    c.ms_set_state(x0, v0)
    assert _code(c.ms_step, s["dt"], max_backtracks=0) == ms.MS_E_LINESEARCH
    x, v = c.ms_get_state()
    assert np.array_equal(x, x0) and np.array_equal(v, v0)
    c.ms_step(s["dt"])
    x, _ = c.ms_get_state()
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    xo, _, _ = newton.newton_step(body, x0, v0, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](1))
    err = e_rel(x, xo, x0)
    say("squashed cube after a failed step: e_rel", err)
    assert err <= 1e-6
    c.close()


def test_failed_step_keeps_the_bdf2_history(dev):
    """A BDF2 step that fails (Newton capped at one iteration: MS_E_NOCONV)
    leaves x, v and the previous step's history untouched: redoing it gives
    bitwise the states of a context that never failed."""
    from paper_2508_13386_amd import ms
    s, x0 = _squashed(3)
    runs = []
    for fail_first in (False, True):
        c = ms.context_from_scene(dev, s)
        c.ms_set_state(x0, np.zeros_like(x0))
        c.ms_step(s["dt"], integrator=1)  # implicit Euler (no history yet)
        x1, v1 = c.ms_get_state()
        if fail_first:
            assert _code(c.ms_step, s["dt"], integrator=1, max_newton=1) == ms.MS_E_NOCONV
            x, v = c.ms_get_state()
            assert np.array_equal(x, x1) and np.array_equal(v, v1)
        c.ms_step(s["dt"], integrator=1)  # BDF2 with the history of step 1
        runs.append(c.ms_get_state())
        c.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
