"""Pins of the oracle's Newton timestep with IPC self-contact: the box
filter of the constraint set, the CCD bound along a step, the assembled
gradient and Hessian of the step energy against central differences, and
momentum conservation when two free bodies collide."""
import numpy as np
import pytest
import torch

import scenes
from oracle import fem, newton
from oracle import selfcontact as sc


def _scene(**kw):
    s = scenes.stacked_cubes(N=2, **kw)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    return s, body, sc.surface(s["tets"])


def _min_pair_distance(x, surf, pairs):
    d = []
    for kind, lst in (("pt", pairs[0]), ("ee", pairs[1])):
        f = sc.pt_dist2 if kind == "pt" else sc.ee_dist2
        for q in lst:
            d.append(float(f(torch.tensor(x[list(q)].ravel(), dtype=torch.float64))))
    return np.sqrt(min(d)) if d else np.inf


def test_filtered_constraint_set_equals_brute_force():
    s, body, surf = _scene()
    dhat = s["selfcontact"]["dhat"]
    x = s["x0"].copy()
    x[s["n_lower"]:, 2] -= 0.6e-3  # the 1e-3 gap closes to 0.2 d_hat
    brute = sc.active_pairs(x, surf, dhat)
    fast = sc.active_pairs_filtered(x, surf, dhat)
    assert sorted(brute[0]) == sorted(fast[0]) and sorted(brute[1]) == sorted(fast[1])
    assert len(brute[0]) > 0 and len(brute[1]) > 0


def test_ccd_bound_stops_before_any_impact():
    s, body, surf = _scene()
    x = s["x0"]
    d = np.zeros_like(x)
    d[s["n_lower"]:, 2] = -0.05  # would push the upper cube deep into the lower one
    t = sc.ccd_bound(x, d, surf)
    assert 0.0 < t < 1.0
    # no pair of the surface touches anywhere on [0, t]
    allp = sc.candidate_pairs(x, surf, 0.0, x + d)
    for tau in np.linspace(0.0, t, 21):
        assert _min_pair_distance(x + tau * d, surf, allp) > 0.0
    # and the bound is not vacuous: the impact itself is not far beyond it
    gap = s["x0"][s["n_lower"]:, 2].min() - s["x0"][:s["n_lower"], 2].max()
    assert t <= gap / 0.05


def test_step_gradient_and_hessian_match_finite_differences():
    s, body, surf = _scene()
    dhat = s["selfcontact"]["dhat"]
    x = s["x0"].copy()
    x[s["n_lower"]:, 2] -= 0.5e-3  # the 1e-3 gap closes to d_hat / 4
    prob = fem.StepProblem(body, s["x0"], s["v0"], s["dt"], s["gravity"], selfcontact=s["selfcontact"])
    pairs = sc.active_pairs_filtered(x, surf, dhat)
    assert len(pairs[0]) + len(pairs[1]) > 0
    g = prob.gradient(x).ravel()
    H = prob.hessian(x, project=False)
    # coordinates of vertices in contact pairs: both bodies, every axis
    verts = sorted({v for lst in pairs for q in lst for v in q})
    rng = np.random.default_rng(0)
    pick = rng.choice(verts, size=6, replace=False)
    h = 1e-7
    for v in pick:
        for i in range(3):
            k = 3 * v + i
            xp, xm = x.copy(), x.copy()
            xp[v, i] += h
            xm[v, i] -= h
            fd = (prob.energy(xp) - prob.energy(xm)) / (2 * h)
            assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (v, i, fd, g[k])
            col = (prob.gradient(xp).ravel() - prob.gradient(xm).ravel()) / (2 * h)
            ref = np.asarray(H[:, k].todense()).ravel()
            assert np.abs(col - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max()), (v, i)


def test_collision_of_free_bodies_conserves_momentum_and_separation():
    s, body, surf = _scene(free=True, speed=0.3)
    x, v = s["x0"], s["v0"]
    p0 = (body.mass[:, None] * v).sum(axis=0)
    scale = np.abs(body.mass[:, None] * v).sum()
    touched = False
    for k in range(1, 3):
        x, v, _ = newton.newton_step(body, x, v, s["dt"], s["gravity"], selfcontact=s["selfcontact"])
        p = (body.mass[:, None] * v).sum(axis=0)
        assert np.allclose(p, p0, rtol=0, atol=1e-10 * scale)
        pairs = sc.active_pairs_filtered(x, surf, s["selfcontact"]["dhat"])
        if pairs[0] or pairs[1]:
            touched = True
            assert _min_pair_distance(x, surf, pairs) > 0.0
    assert touched
    # the bodies were pushed apart: the approach speed dropped
    vz = v[:, 2]
    assert vz[s["n_lower"]:].mean() - vz[:s["n_lower"]].mean() > -0.6
