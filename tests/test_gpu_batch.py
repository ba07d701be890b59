"""Batched timesteps of several uneven scenes in one set of launches: every
scene equals its own unbatched ms_step run (same arithmetic, so the states
agree bitwise), across consecutive steps that reuse the cached union."""
import numpy as np
import pytest

import scenes
from tests.gpu_util import device, say

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
    for step in range(1, 3):
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
    with pytest.raises(ms.MSError) as e:
        ms.ms_batch_step(bat, scs[0]["dt"])
    assert e.value.code == ms.MS_E_ARG
    for c in bat:
        c.close()
