"""Pins of the paper-mode oracle (Alg. 1 and 2): the PCG stop rule of the
subspace solves, the block-Jacobi and Jacobi preconditioners, the Hessian-lag
trigger, the refinement count from the partitions' hop diameters, and
convergence to the exact minimiser when every level is solved to completion."""
import numpy as np
import pytest

import scenes
from oracle import basis as obasis
from oracle import fem, newton, paper


def _block_partition(rest, tets, k):
    c = rest[tets].mean(axis=1)
    lo, hi = rest.min(axis=0), rest.max(axis=0)
    idx = np.minimum((k * (c - lo) / (hi - lo)).astype(int), k - 1)
    return idx[:, 0] * k * k + idx[:, 1] * k + idx[:, 2]


def _basis(s, k=2):
    rest, tets = s["rest"], s["tets"]
    part = _block_partition(rest, tets, k)
    out = obasis.basis_weights(rest, tets, s["E"], s["dirichlet"], part)
    vptr = np.zeros(len(rest) + 1, np.int64)
    vptr[1:] = np.cumsum([len(r) for r in out["rows"]])
    return dict(origins=out["origins"], vptr=vptr, m=len(out["origins"]), part=part,
                vhandle=np.array([i for r in out["rows"] for i, _ in r], np.int32),
                vphi=np.array([p for r in out["rows"] for _, p in r]))


def _spd(N, rng, cond=1e6):
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    return (Q * np.geomspace(1.0, cond, N)) @ Q.T


# -- PCG stop rule and preconditioners ---------------------------------------

def test_subspace_pcg_stops_at_rtol_and_not_earlier():
    rng = np.random.default_rng(7)
    N = 12 * 6
    A = _spd(N, rng)
    b = rng.standard_normal(N)
    x, k = paper.block_pcg(A, b, 1e-4)
    assert k >= 5
    # the returned iterate meets the rule (true residual; the recursive one
    # it is tested on agrees to round-off) ...
    assert np.linalg.norm(b - A @ x) <= 1e-4 * np.linalg.norm(b) * (1 + 1e-6)
    # ... and the iterate one step earlier does not
    x1, k1 = paper.pcg(A, b, paper.block_jacobi_dense(A, 12), 1e-4, k - 1)
    assert k1 == k - 1
    assert np.linalg.norm(b - A @ x1) > 1e-4 * np.linalg.norm(b)
    # a zero right-hand side takes no iteration
    x0, k0 = paper.block_pcg(A, np.zeros(N), 1e-4)
    assert k0 == 0 and not x0.any()


def test_block_diagonal_system_takes_one_iteration():
    """With A block diagonal in 12 x 12 blocks the block-Jacobi preconditioner
    is A^-1 itself: one iteration gives the solution (the single-object
    affine level of Alg. 2 is such a system)."""
    rng = np.random.default_rng(3)
    blocks = [_spd(12, rng, 1e4) for _ in range(5)]
    A = np.zeros((60, 60))
    for k, B in enumerate(blocks):
        A[12 * k:12 * k + 12, 12 * k:12 * k + 12] = B
    b = rng.standard_normal(60)
    x, k = paper.block_pcg(A, b, 1e-12)
    assert k == 1
    assert np.abs(x - np.linalg.solve(A, b)).max() <= 1e-10 * np.abs(np.linalg.solve(A, b)).max()


def test_block_jacobi_leaves_null_handles_at_zero():
    """A handle with no free vertex has a zero 12 x 12 block and zero
    right-hand side entries; the PCG solution is zero there and solves the
    rest of the system."""
    rng = np.random.default_rng(4)
    A = _spd(36, rng, 1e3)
    A[12:24, :] = 0.0
    A[:, 12:24] = 0.0
    b = rng.standard_normal(36)
    b[12:24] = 0.0
    x, _ = paper.block_pcg(A, b, 1e-13)
    keep = np.r_[0:12, 24:36]
    assert not x[12:24].any()
    ref = np.linalg.solve(A[np.ix_(keep, keep)], b[keep])
    assert np.abs(x[keep] - ref).max() <= 1e-8 * np.abs(ref).max()


def test_block_generalised_inverse():
    """ldl_pinv is the inverse of a nonsingular SPD block and a generalised
    inverse (B X B = B, X symmetric) of a rank-deficient PSD one, such as the
    block of a handle whose free vertices are coplanar."""
    rng = np.random.default_rng(5)
    B = _spd(12, rng, 1e6)
    assert np.abs(paper.ldl_pinv(B) @ B - np.eye(12)).max() <= 1e-8
    Y = rng.standard_normal((12, 9))
    Bs = Y @ Y.T  # rank 9
    X = paper.ldl_pinv(Bs)
    assert np.abs(Bs @ X @ Bs - Bs).max() <= 1e-10 * np.abs(Bs).max()
    assert np.abs(X - X.T).max() <= 1e-12 * np.abs(X).max()
    assert not paper.ldl_pinv(np.zeros((12, 12))).any()


def test_refinement_jacobi_pcg():
    rng = np.random.default_rng(1)
    # diagonal system: the Jacobi preconditioner is exact after one iteration
    d = rng.uniform(1.0, 100.0, 30)
    b = rng.standard_normal(30)
    x1 = paper.jacobi_pcg(np.diag(d), b, 1)
    assert np.abs(x1 - b / d).max() <= 1e-14 * np.abs(b / d).max()
    # the preconditioner is the diagonal, not the 3x3 blocks: a matrix whose
    # diagonal blocks are not diagonal needs more than one iteration
    A = np.kron(np.eye(10), np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]]))
    xa = paper.jacobi_pcg(A, b, 1)
    assert np.linalg.norm(b - A @ xa) > 1e-3 * np.linalg.norm(b)
    # run to N iterations on a general SPD matrix: the direct solve
    N = 30
    M = rng.standard_normal((N, N))
    M = M @ M.T + N * np.eye(N)
    x = paper.jacobi_pcg(M, b, N)
    ref = np.linalg.solve(M, b)
    assert np.abs(x - ref).max() <= 1e-8 * np.abs(ref).max()
    # fewer iterations: a residual strictly smaller than the initial one
    x5 = paper.jacobi_pcg(M, b, 5)
    assert np.linalg.norm(b - M @ x5) < np.linalg.norm(b)


# -- Hessian-lag trigger --------------------------------------------------------

def _schedule(seq, window, threshold, gap):
    alphas, last, out = [], -10 ** 9, []
    for it, a in enumerate(seq):
        if paper.lag_should_refresh(it, alphas, last, window, threshold, gap):
            last = it
            out.append(it)
        alphas.append(a)
    return out


def test_lag_trigger_on_a_scripted_step_sequence():
    """Worked out by hand: refresh at the step start; then the mean of the last
    three accepted steps must be below 0.5 and five iterations must have passed
    since the last refresh.  At 5 the mean of steps 2-4 is 0.25; 6-9 are too
    close to 5; at 10 and 11 the means are 1 and 0.7; at 12 it is 0.4."""
    seq = [1, .25, .25, .25, .25, .25, .25, 1, 1, 1, .1, .1, .1, .1]
    assert _schedule(seq, 3, 0.5, 5) == [0, 5, 12]
    # without the gap rule: not at 3 (steps 0-2 average exactly 0.5, which
    # is not below it), then at 4-7 (0.25); at 8 steps 5-7 average 0.5 again,
    # at 9-11 0.75, 1 and 0.7; at 12 and 13 0.4 and 0.1
    assert _schedule(seq, 3, 0.5, 1) == [0, 4, 5, 6, 7, 12, 13]
    # a window of one and threshold 0.2: only after the first 0.1 step
    assert _schedule(seq, 1, 0.2, 5) == [0, 11]


def test_paper_step_follows_the_lag_trigger():
    s = scenes.inclusion_block(4, seed=0, steps=1)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    B = _basis(s)
    rec = []
    paper.paper_step(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](1), None, B,
                     refine_iters=20, record=rec, threshold=0.99, gap=2)
    alphas = [r["alpha"] for r in rec]
    expect = _schedule(alphas, 3, 0.99, 2)
    assert [i for i, r in enumerate(rec) if r["refresh"]] == expect


# -- refinement count from the partitions' hop diameters ------------------------

def _kuhn_hops(d):
    """Graph distance of the Kuhn (Freudenthal) lattice: its edges are the
    vectors with entries all in {0, 1} or all in {0, -1}, so a displacement
    needs max(positive parts) steps of the first kind plus max(negative
    parts) of the second."""
    d = np.asarray(d)
    return np.maximum(d, 0).max(axis=-1) + np.maximum(-d, 0).max(axis=-1)


@pytest.mark.parametrize("N,k,expect_iters", [(8, 2, 20), (32, 1, 40)])
def test_hop_rule_on_kuhn_blocks(N, k, expect_iters):
    rest, tets, _, _ = scenes.kuhn_cube(N)
    part = _block_partition(rest, tets, k)
    origins = np.array([rest[np.unique(tets[part == l])].mean(axis=0) for l in range(k ** 3)])
    diam = paper.partition_hop_diameters(rest, tets, part, origins)
    # each block of N/k cells is centred on a vertex; the farthest vertices
    # are the corners of mixed sign, (N/k)/2 + (N/k)/2 hops away
    g = np.rint(rest * N).astype(int)
    for l in range(k ** 3):
        verts = np.unique(tets[part == l])
        centre = np.rint(origins[l] * N).astype(int)
        assert diam[l] == _kuhn_hops(g[verts] - centre).max() == N // k
    iters, mean = paper.refine_iterations(rest, tets, part, origins)
    assert mean == N // k and iters == expect_iters


# -- the three levels together ---------------------------------------------------

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
    scale = np.abs(g).max()
    # solved to completion: the affine correction leaves no residual in the
    # affine space, and the sparse level none in the (larger) sparse space
    da, ds, ia, is_ = paper.subspace_direction(H, g, Ua, Us, rtol=1e-14)
    assert ia == 1  # one object: one 12 x 12 block
    assert np.abs(Ua.T @ (H @ da + g)).max() <= 1e-9 * scale * np.abs(Ua).max()
    assert np.abs(Us.T @ (H @ ds + g)).max() <= 1e-9 * scale * np.abs(Us).max()
    # to the paper's 1e-4: the sparse-level residual is within 1e-4 of its
    # right-hand side
    da4, ds4, _, is4 = paper.subspace_direction(H, g, Ua, Us, rtol=1e-4)
    rhs = Us.T @ (-g - H @ da4)
    assert np.linalg.norm(Us.T @ (-g - H @ ds4)) <= 1e-4 * np.linalg.norm(rhs) * (1 + 1e-6)
    assert 1 <= is4 < is_
    # the sparse space contains the affine one (partition of unity)
    coef = np.linalg.lstsq(Us, Ua, rcond=None)[0]
    assert np.abs(Us @ coef - Ua).max() <= 1e-10


def test_fully_solved_levels_reach_the_exact_minimiser():
    """With a tight subspace decrement, subspace solves to round-off and a
    refinement solved to completion the three-level iteration is a Newton
    method on E and must land on the oracle's exact minimiser."""
    s = scenes.plain_cube(3, seed=5)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    B = _basis(s)
    x_ref, _, _ = newton.newton_step(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"],
                                     s["dbc_targets"](1))
    x, _, info = paper.paper_step(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"],
                                  s["dbc_targets"](1), None, B, eps=1e-13, refine_iters=3 * len(s["rest"]),
                                  rtol=1e-14)
    e = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref - s["x0"])
    assert e <= 1e-6, e
    assert info["refreshes"] >= 1
