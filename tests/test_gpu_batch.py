"""Batched timesteps of several uneven scenes in one set of launches: every
scene equals its own unbatched ms_step run (same arithmetic, so the states
agree bitwise), across consecutive steps that reuse the cached union."""
import numpy as np
import pytest

import scenes
from oracle import fem, newton
from tests.gpu_util import device, e_rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _contexts(dev, scs):
    from paper_2508_13386_amd import ms
    return [ms.context_from_scene(dev, s) for s in scs]


@pytest.mark.parametrize("prec_name,forcing", [("fp64", 0), ("mixed", 1)])
def test_batch_equals_unbatched(dev, prec_name, forcing):
    from paper_2508_13386_amd import ms
    prec = ms.PREC_MIXED if prec_name == "mixed" else ms.PREC_FP64
    scs = scenes.batch_scenes(5, seed=7, t_lo=300, t_hi=4000)
    say("batch sizes", [len(s["tets"]) for s in scs], prec_name)
    ref = _contexts(dev, scs)
    bat = _contexts(dev, scs)
    dt = scs[0]["dt"]
    bodies = [fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"]) for s in scs]
    for step in range(1, 3):
        starts = [c.ms_get_state() for c in bat]
        st_ref = [c.ms_step(dt, precision=prec, forcing=forcing) for c in ref]
        st_bat = ms.ms_batch_step(bat, dt, precision=prec, forcing=forcing)
        for q, (cr, cb) in enumerate(zip(ref, bat)):
            xr, vr = cr.ms_get_state()
            xb, vb = cb.ms_get_state()
            u = np.linalg.norm(xr - scs[q]["rest"])
            diff = np.abs(xr - xb).max()
            say("step", step, "scene", q, "newton", st_ref[q]["newton_iters"], st_bat[q]["newton_iters"], "pcg",
                st_ref[q]["pcg_iters"], st_bat[q]["pcg_iters"], "max |dx|", diff, "|u|", u)
            assert st_ref[q]["newton_iters"] == st_bat[q]["newton_iters"]
            assert st_ref[q]["pcg_iters"] == st_bat[q]["pcg_iters"]
            assert np.array_equal(xr, xb) and np.array_equal(vr, vb)
            # and each batched scene reaches the oracle's minimiser from the same state
            x0, v0 = starts[q]
            sc = scs[q]
            xo, _, _ = newton.newton_step(bodies[q], x0, v0, dt, sc["gravity"], sc["dirichlet"],
                                          sc["dbc_targets"](step))
            err = e_rel(xb, xo, x0)
            say("   scene", q, "batched vs oracle e_rel", err)
            assert err <= 1e-6
    for c in ref + bat:
        c.close()


@pytest.mark.parametrize("prec_name,coarse_move", [("fp64", 0.2), ("mixed", 0.2), ("mixed", 0.0)])
def test_batch_two_level_equals_unbatched(dev, prec_name, coarse_move):
    """The additive two-level preconditioner in a batch: each scene keeps its
    own basis, coarse matrix and inverse (formed from its segment of the
    union's Hessian, on its own rebuild rule), the union carries the
    scenes' transfer operators, and a block-diagonal GEMV applies the
    inverses.  Every scene equals its own ms_step bitwise (states, PCG and
    Newton counts, coarse rebuilds) and reaches the oracle's minimiser."""
    from paper_2508_13386_amd import ms
    prec = ms.PREC_MIXED if prec_name == "mixed" else ms.PREC_FP64
    scs = scenes.batch_scenes(4, seed=5, t_lo=500, t_hi=4000)
    say("two-level batch sizes", [len(s["tets"]) for s in scs], prec_name, "coarse_move", coarse_move)
    ref = _contexts(dev, scs)
    bat = _contexts(dev, scs)
    for c in ref + bat:
        c.ms_build_basis(n_handles=6, seed=2)
    params = ms.solver_defaults(precision=prec, preconditioner=ms.PC_TWO_LEVEL_ADDITIVE, forcing=1,
                                pcg_eta_max=0.1, pcg_eta_min=1e-4, coarse_move=coarse_move)
    dt = scs[0]["dt"]
    bodies = [fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"]) for s in scs]
    for step in range(1, 3):
        starts = [c.ms_get_state() for c in bat]
        st_ref = [c.ms_step(dt, params) for c in ref]
        st_bat = ms.ms_batch_step(bat, dt, params)
        for q in range(len(scs)):
            xr, vr = ref[q].ms_get_state()
            xb, vb = bat[q].ms_get_state()
            x0, v0 = starts[q]
            sc = scs[q]
            xo, _, _ = newton.newton_step(bodies[q], x0, v0, dt, sc["gravity"], sc["dirichlet"],
                                          sc["dbc_targets"](step))
            err = e_rel(xb, xo, x0)
            say("step", step, "scene", q, "newton", st_ref[q]["newton_iters"], st_bat[q]["newton_iters"], "pcg",
                st_ref[q]["pcg_iters"], st_bat[q]["pcg_iters"], "rebuilds", st_ref[q]["hessian_refreshes"],
                st_bat[q]["hessian_refreshes"], "max |dx|", float(np.abs(xr - xb).max()), "oracle e_rel", err)
            assert st_ref[q]["pcg_iters"] == st_bat[q]["pcg_iters"]
            assert st_ref[q]["hessian_refreshes"] == st_bat[q]["hessian_refreshes"]
            assert np.array_equal(xr, xb) and np.array_equal(vr, vb)
            assert err <= 1e-6
    for c in ref + bat:
        c.close()


@pytest.mark.parametrize("pc_name", ["jacobi", "additive"])
def test_batch_contact_equals_unbatched(dev, pc_name):
    """Half-space contact in a batch: gyroid spheres of three resolutions
    dropped onto the slab (one shared half-space; the barrier stiffness set
    equal), each scene's line search starting from its own CCD bound.  Every
    scene equals its own ms_step bitwise and reaches the oracle's
    minimiser; the first steps bring the spheres into the barrier's range."""
    from paper_2508_13386_amd import ms
    scs = [scenes.gyroid_sphere(res=r) for r in (8, 10, 12)]
    kappa = scs[1]["halfspace"]["kappa"]
    for sc in scs:
        sc["halfspace"] = dict(sc["halfspace"], kappa=kappa)
    say("contact batch", [len(sc["tets"]) for sc in scs], pc_name)
    ref = _contexts(dev, scs)
    bat = _contexts(dev, scs)
    pc = ms.PC_BLOCK_JACOBI
    if pc_name == "additive":
        pc = ms.PC_TWO_LEVEL_ADDITIVE
        for c in ref + bat:
            c.ms_build_basis(n_handles=6, seed=2)
    params = ms.solver_defaults(precision=ms.PREC_MIXED, preconditioner=pc, forcing=1, pcg_eta_max=0.1,
                                pcg_eta_min=1e-4, coarse_move=0.2)
    dt = scs[0]["dt"]
    bodies = [fem.Body(sc["rest"], sc["tets"], sc["E"], sc["nu"], sc["rho"]) for sc in scs]
    b = ms.Batch(bat)
    for step in range(1, 4):
        starts = [c.ms_get_state() for c in bat]
        st_ref = [c.ms_step(dt, params) for c in ref]
        st_bat = b.advance(dt, params)
        for q, sc in enumerate(scs):
            xr, vr = ref[q].ms_get_state()
            xb, vb = bat[q].ms_get_state()
            x0, v0 = starts[q]
            xo, _, _ = newton.newton_step(bodies[q], x0, v0, dt, sc["gravity"], sc["dirichlet"],
                                          sc["dbc_targets"](step), halfspace=sc["halfspace"])
            err = e_rel(xb, xo, x0)
            gap = float(xb[:, 2].min())
            say("step", step, "scene", q, "newton", st_ref[q]["newton_iters"], st_bat[q]["newton_iters"], "pcg",
                st_ref[q]["pcg_iters"], st_bat[q]["pcg_iters"], "min alpha", st_bat[q]["min_alpha"],
                "lowest z", gap, "oracle e_rel", err)
            assert np.array_equal(xr, xb) and np.array_equal(vr, vb)
            assert err <= 1e-6
    assert min(float(c.ms_get_state()[0][:, 2].min()) for c in bat) < scs[0]["halfspace"]["dhat"]
    b.close()
    for c in ref + bat:
        c.close()


def test_created_batch_equals_unbatched(dev):
    """ms_batch_create / ms_batch_advance: the union built once, stepped
    three times, equals each context's own ms_step bitwise; a context whose
    mesh changed after creation is refused."""
    from paper_2508_13386_amd import ms
    scs = scenes.batch_scenes(4, seed=11, t_lo=300, t_hi=3000)
    ref = _contexts(dev, scs)
    bat = _contexts(dev, scs)
    b = ms.Batch(bat)
    dt = scs[0]["dt"]
    for step in range(1, 4):
        st_ref = [c.ms_step(dt, precision=ms.PREC_MIXED, forcing=1) for c in ref]
        st_bat = b.advance(dt, precision=ms.PREC_MIXED, forcing=1)
        for q in range(len(scs)):
            xr, vr = ref[q].ms_get_state()
            xb, vb = bat[q].ms_get_state()
            say("created batch step", step, "scene", q, "pcg", st_ref[q]["pcg_iters"], st_bat[q]["pcg_iters"])
            assert np.array_equal(xr, xb) and np.array_equal(vr, vb)
    with pytest.raises(ms.MSError) as e:
        b.advance(dt, mode=ms.MODE_PAPER)
    assert e.value.code == ms.MS_E_ARG
    b.close()
    for c in ref + bat:
        c.close()


def test_batch_rejects_unsupported(dev):
    from paper_2508_13386_amd import ms
    scs = scenes.batch_scenes(2, seed=3, t_lo=300, t_hi=600)
    bat = _contexts(dev, scs)
    with pytest.raises(ms.MSError) as e:
        ms.ms_batch_step(bat, scs[0]["dt"], mode=ms.MODE_PAPER)
    assert e.value.code == ms.MS_E_ARG
    g = scenes.gyroid_sphere(res=8)
    bat.append(ms.context_from_scene(dev, g))
    with pytest.raises(ms.MSError) as e:  # scenes with and without a half-space
        ms.ms_batch_step(bat, scs[0]["dt"])
    assert e.value.code == ms.MS_E_ARG
    for c in bat:
        c.close()
