"""Pins of the cubature oracle (Sec. 3.8, modal moment fitting; Alg. 3)."""
import numpy as np
import pytest
import scipy.sparse as sp

import scenes
from oracle import basis as obasis
from oracle import cubature as cub
from oracle import fem, linops, paper


def _partition(rest, tets, k=2):
    c = rest[tets].mean(axis=1)
    lo, hi = rest.min(axis=0), rest.max(axis=0)
    idx = np.minimum((k * (c - lo) / (hi - lo)).astype(int), k - 1)
    return idx[:, 0] * k * k + idx[:, 1] * k + idx[:, 2]


def _basis(s, part):
    out = obasis.basis_weights(s["rest"], s["tets"], s["E"], s["dirichlet"], part)
    vptr = np.zeros(len(s["rest"]) + 1, np.int64)
    vptr[1:] = np.cumsum([len(r) for r in out["rows"]])
    return dict(origins=out["origins"], vptr=vptr, m=len(out["origins"]), part=np.asarray(part),
                vhandle=np.array([i for r in out["rows"] for i, _ in r], np.int32),
                vphi=np.array([p for r in out["rows"] for _, p in r]))


def _brute_moments(rest, tets, part, basis, p, wfull):
    """(cubature sums, exact sums) of 1, u_i, u_i u_j over partition p, by
    loops over elements and vertices (no shared helper with the oracle)."""
    phi = [dict() for _ in range(len(rest))]
    for v in range(len(rest)):
        for k in range(basis["vptr"][v], basis["vptr"][v + 1]):
            phi[v][int(basis["vhandle"][k])] = phi[v].get(int(basis["vhandle"][k]), 0.0) + basis["vphi"][k]
    elems = [e for e in range(len(tets)) if part[e] == p]
    hs = sorted({i for e in elems for v in tets[e] for i, val in phi[v].items() if val != 0.0})
    got, ref = {}, {}
    for e in elems:
        X = rest[tets[e]]
        vol = abs(np.linalg.det(np.array([X[1] - X[0], X[2] - X[0], X[3] - X[0]]).T)) / 6.0
        u = {i: sum(phi[v].get(i, 0.0) for v in tets[e]) / 4.0 for i in hs}
        terms = {(): 1.0}
        for i in hs:
            terms[(i,)] = u[i]
        for a in hs:
            for b in hs:
                if a <= b:
                    terms[(a, b)] = u[a] * u[b]
        for key, val in terms.items():
            ref[key] = ref.get(key, 0.0) + vol * val
            got[key] = got.get(key, 0.0) + wfull[e] * val
    keys = sorted(ref)
    return np.array([got[k] for k in keys]), np.array([ref[k] for k in keys])


def test_splitmix64_published_outputs():
    # the reference generator from state 0 (state advanced by gamma before mixing)
    outs = [cub.splitmix64((k * cub.GAMMA) & cub.MASK64) for k in (1, 2, 3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = np.array([cub.uniform(7, j) for j in range(2000)])
    assert u.min() >= 0.0 and u.max() < 1.0 and len(np.unique(u)) == len(u)
    assert abs(u.mean() - 0.5) < 0.03


def test_moment_system_matches_brute_force_and_full_selection_is_exact():
    s = scenes.plain_cube(4, seed=1)
    part = _partition(s["rest"], s["tets"])
    B = _basis(s, part)
    vol = cub.tet_volumes(s["rest"], s["tets"])
    assert vol.sum() == pytest.approx(1.0, rel=1e-12)
    Ue = cub.element_values(s["tets"], B["vptr"], B["vhandle"], B["vphi"], B["m"])
    for p in np.unique(part):
        ids = np.nonzero(part == p)[0]
        A, b, touch = cub.moment_system(Ue[ids], vol[ids])
        k = len(touch)
        assert A.shape == (1 + k + k * (k + 1) // 2, len(ids))
        got, ref = _brute_moments(s["rest"], s["tets"], part, B, p, vol)
        assert np.sort(b) == pytest.approx(np.sort(ref), rel=1e-12, abs=1e-15)
        assert b[0] == pytest.approx(vol[ids].sum(), rel=1e-14)
        # every element with its own volume: the conditions hold exactly
        assert np.linalg.norm(A @ vol[ids] - b) <= 1e-14 * np.linalg.norm(b)


def test_fit_reaches_tolerance_with_sparse_nonnegative_weights():
    s = scenes.plain_cube(4, seed=2)
    part = _partition(s["rest"], s["tets"])
    B = _basis(s, part)
    t, w, res = cub.fit_cubature(s["rest"], s["tets"], part, B, seed=3, n_init=8, n_add=8, tol=1e-9)
    assert np.all(w > 0.0) and len(np.unique(t)) == len(t)
    assert len(t) < len(s["tets"])
    wfull = np.zeros(len(s["tets"]))
    wfull[t] = w
    Ue = cub.element_values(s["tets"], B["vptr"], B["vhandle"], B["vphi"], B["m"])
    for p in np.unique(part):
        got, ref = _brute_moments(s["rest"], s["tets"], part, B, p, wfull)
        assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)
        assert res[int(p)] <= 1e-9
        # NNLS returns a basic solution: no more points than moment conditions
        ids = np.nonzero(part == p)[0]
        A, _, _ = cub.moment_system(Ue[ids], np.ones(len(ids)))
        assert np.count_nonzero(part[t] == p) <= np.linalg.matrix_rank(A)
    assert cub.moment_residuals(s["rest"], s["tets"], part, B, t, w) == pytest.approx(res, abs=1e-12)


def test_single_constant_function_needs_one_point():
    # one basis function equal to 1 everywhere: every moment row is the same
    # (rank one), so one element carrying the partition volume suffices
    s = scenes.plain_cube(3, seed=0)
    n = len(s["rest"])
    part = _partition(s["rest"], s["tets"])
    B = dict(m=1, vptr=np.arange(n + 1), vhandle=np.zeros(n, np.int32), vphi=np.ones(n))
    vol = cub.tet_volumes(s["rest"], s["tets"])
    t, w, res = cub.fit_cubature(s["rest"], s["tets"], part, B, seed=1, n_init=4, n_add=4)
    for p in np.unique(part):
        sel = part[t] == p
        assert sel.sum() == 1
        assert w[sel][0] == pytest.approx(vol[part == p].sum(), rel=1e-12)


def _contact_state(s, seed):
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    rng = np.random.default_rng(seed)
    x = s["x0"] + 0.002 * rng.standard_normal(s["x0"].shape)
    return body, x


@pytest.mark.parametrize("name", ["plain", "sliding"])
def test_full_selection_galerkin_is_the_galerkin_matrix(name):
    s = scenes.plain_cube(3, seed=4) if name == "plain" else scenes.sliding_cube(3)
    body, x = _contact_state(s, 5)
    if s["halfspace"] is not None:
        x[:, 2] = np.maximum(x[:, 2], 2e-4)  # inside the barrier's range, off the plane
    part = _partition(s["rest"], s["tets"])
    B = _basis(s, part)
    pinned = np.zeros(len(x), bool)
    pinned[s["dirichlet"]] = True
    Us, _ = paper.basis_matrices(body, B, pinned)
    prob = fem.StepProblem(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["halfspace"])
    fm = sp.diags(np.repeat(~pinned, 3).astype(np.float64))
    H = (fm @ prob.hessian(x) @ fm).tocsr()
    K_ref = linops.galerkin(Us, H)
    K = cub.cubature_galerkin(prob, x, Us, np.arange(len(s["tets"])), body.vol)
    assert np.abs(K - K_ref).max() <= 1e-12 * np.abs(K_ref).max()
    # a fitted cubature keeps the matrix symmetric positive semi-definite
    t, w, _ = cub.fit_cubature(s["rest"], s["tets"], part, B, seed=2, n_init=8, n_add=8)
    Kc = cub.cubature_galerkin(prob, x, Us, t, w)
    assert np.abs(Kc - Kc.T).max() <= 1e-13 * np.abs(Kc).max()
    assert np.linalg.eigvalsh(Kc).min() >= -1e-12 * np.abs(Kc).max()


def test_paper_step_with_full_selection_cubature_is_the_exact_paper_step():
    s = scenes.plain_cube(3, seed=6)
    part = _partition(s["rest"], s["tets"])
    B = _basis(s, part)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    tgt = s["dbc_targets"](1)
    args = (body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"], tgt, None, B)
    x0, _, i0 = paper.paper_step(*args)
    x1, _, i1 = paper.paper_step(*args, cubature=(np.arange(len(s["tets"])), body.vol))
    assert i0["newton"] == i1["newton"]
    # the two subspace matrices agree to round-off; through the iterative
    # subspace solves that reaches the positions as a few ulps of x
    assert np.abs(x1 - x0).max() <= 1e-12 * np.abs(x0 - s["x0"]).max() + 8 * np.finfo(float).eps * np.abs(x0).max()
    # a fitted cubature changes the step only slightly (an approximation)
    t, w, _ = cub.fit_cubature(s["rest"], s["tets"], part, B, seed=1, n_init=8, n_add=8)
    x2, _, _ = paper.paper_step(*args, cubature=(t, w))
    assert np.abs(x2 - x0).max() <= 0.5 * np.abs(x0 - s["x0"]).max()
