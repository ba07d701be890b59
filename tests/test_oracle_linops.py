"""Pins of the oracle's operator definitions against explicit loops."""
import numpy as np

import scenes
from oracle import linops


def test_bsr_matvec_matches_loops():
    rp, col, vals = scenes.spd_bsr_pattern(3, seed=1)
    n = len(rp) - 1
    x = np.random.default_rng(0).standard_normal((n, 3))
    y = linops.bsr_matvec(rp, col, vals, x)
    ref = np.zeros((n, 3))
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            ref[i] += vals[k] @ x[col[k]]
    assert np.allclose(y, ref, rtol=0, atol=1e-12)


def test_dense_basis_reproduces_affine_fields():
    """With phi a partition of unity, setting every handle to the same affine
    map A reproduces A exactly (linear precision of Eq. LBS with POU)."""
    rest, _, _, _ = scenes.kuhn_cube(3)
    n, m = len(rest), 4
    rng = np.random.default_rng(1)
    origins = rng.uniform(0, 1, (m, 3))
    W = rng.uniform(0, 1, (n, m)) * (rng.uniform(size=(n, m)) < 0.6)
    W[:, 0] += 1e-3
    W /= W.sum(axis=1, keepdims=True)
    vptr = np.concatenate([[0], np.cumsum((W > 0).sum(axis=1))])
    vh = np.concatenate([np.nonzero(w > 0)[0] for w in W])
    vphi = W[W > 0]
    U = linops.dense_basis(rest, origins, vptr, vh, vphi, m)
    A = rng.standard_normal((3, 3))
    t = rng.standard_normal(3)
    q = np.zeros(12 * m)
    for i in range(m):
        # displacement field u(x) = A x + t written about origin o_i: t + A o_i + A (x - o_i)
        c = t + A @ origins[i]
        for a in range(3):
            q[12 * i + 4 * a:12 * i + 4 * a + 4] = [c[a], *A[a]]
    u = linops.prolong(U, q)
    assert np.allclose(u, rest @ A.T + t, atol=1e-12)


def test_galerkin_and_coarse_solve():
    rng = np.random.default_rng(2)
    U = rng.standard_normal((30, 6))
    M = rng.standard_normal((30, 30))
    H = M @ M.T + 30 * np.eye(30)
    A = linops.galerkin(U, H)
    c = rng.standard_normal(6)
    e = linops.coarse_solve(A, c)
    assert np.allclose(A @ e, c, atol=1e-10)
    assert np.allclose(A, A.T)
