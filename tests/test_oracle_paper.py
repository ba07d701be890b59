"""Pins of the paper-mode oracle (Alg. 1 and 2): the parts, and convergence
to the exact minimiser when every level is solved to completion."""
import numpy as np
import pytest

import scenes
from oracle import basis as obasis
from oracle import fem, newton, paper


def _basis(s, k=2):
    rest, tets = s["rest"], s["tets"]
    c = rest[tets].mean(axis=1)
    lo, hi = rest.min(axis=0), rest.max(axis=0)
    idx = np.minimum((k * (c - lo) / (hi - lo)).astype(int), k - 1)
    part = idx[:, 0] * k * k + idx[:, 1] * k + idx[:, 2]
    out = obasis.basis_weights(rest, tets, s["E"], s["dirichlet"], part)
    vptr = np.zeros(len(rest) + 1, np.int64)
    vptr[1:] = np.cumsum([len(r) for r in out["rows"]])
    return dict(origins=out["origins"], vptr=vptr, m=len(out["origins"]),
                vhandle=np.array([i for r in out["rows"] for i, _ in r], np.int32),
                vphi=np.array([p for r in out["rows"] for _, p in r]))


def test_subspace_levels_are_galerkin_orthogonal():
    s = scenes.plain_cube(4, seed=3)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    B = _basis(s)
    pinned = np.zeros(len(s["rest"]), bool)
    pinned[s["dirichlet"]] = True
    Us, Ua = paper.basis_matrices(body, B, pinned)
    rng = np.random.default_rng(0)
    x = s["rest"] + 0.01 * rng.standard_normal(s["rest"].shape)
    x[pinned] = s["rest"][pinned]
    prob = fem.StepProblem(body, s["x0"], s["v0"], s["dt"], s["gravity"])
    fm = np.repeat(~pinned, 3).astype(float)
    g = prob.gradient(x).ravel() * fm
    H = (np.diag(fm) @ prob.hessian(x).toarray() @ np.diag(fm))
    da, ds = paper.subspace_direction(H, g, Ua, Us)
    scale = np.abs(g).max()
    # the affine correction leaves no residual in the affine space, and the
    # sparse level none in the (larger) sparse space
    assert np.abs(Ua.T @ (H @ da + g)).max() <= 1e-9 * scale * np.abs(Ua).max()
    assert np.abs(Us.T @ (H @ ds + g)).max() <= 1e-9 * scale * np.abs(Us).max()
    # the sparse space contains the affine one (partition of unity)
    coef = np.linalg.lstsq(Us, Ua, rcond=None)[0]
    assert np.abs(Us @ coef - Ua).max() <= 1e-10


def test_refinement_pcg_reaches_the_direct_solve():
    rng = np.random.default_rng(1)
    N = 3 * 10
    A = rng.standard_normal((N, N))
    A = A @ A.T + N * np.eye(N)
    b = rng.standard_normal(N)
    x = paper.block_jacobi_pcg(A, b, N)
    assert np.abs(x - np.linalg.solve(A, b)).max() <= 1e-8 * np.abs(np.linalg.solve(A, b)).max()
    # fewer iterations: a residual strictly smaller than the initial one
    x5 = paper.block_jacobi_pcg(A, b, 5)
    assert np.linalg.norm(b - A @ x5) < np.linalg.norm(b)


def test_fully_solved_levels_reach_the_exact_minimiser():
    """With a tight subspace decrement and a refinement solved to completion
    the three-level iteration is a Newton method on E and must land on the
    oracle's exact minimiser."""
    s = scenes.plain_cube(3, seed=5)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    B = _basis(s)
    x_ref, _, _ = newton.newton_step(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"],
                                     s["dbc_targets"](1))
    x, _, info = paper.paper_step(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"],
                                  s["dbc_targets"](1), None, B, eps=1e-13, refine_iters=3 * len(s["rest"]))
    e = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref - s["x0"])
    assert e <= 1e-6, e
    assert info["refreshes"] >= 1
