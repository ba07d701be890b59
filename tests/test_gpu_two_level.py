"""GPU parity of the two-level preconditioner against dense definitions:
Galerkin U^T H U, restriction / coarse solve / prolongation, and Newton
steps preconditioned by it (relative displacement error <= 1e-6)."""
import numpy as np
import pytest

import scenes
from oracle import fem, linops, newton
from tests.gpu_util import device, e_rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _setup(dev, N=6, m=8, seed=0, scene="inclusion_block"):
    from paper_2508_13386_amd import ms
    s = scenes.inclusion_block(N, seed=seed, steps=3) if scene == "inclusion_block" else scenes.plain_cube(N, seed=seed)
    c = ms.context_from_scene(dev, s)
    c.ms_build_basis(n_handles=m, seed=1)
    return s, c


def _dense_U(s, B):
    U = linops.dense_basis(s["rest"], B["origins"], B["vptr"], B["vhandle"], B["vphi"], B["m"])
    pinned = np.zeros(len(s["rest"]), bool)
    pinned[s["dirichlet"]] = True
    U[np.repeat(pinned, 3)] = 0.0  # the basis vanishes on eliminated DOFs
    return U, pinned


def test_galerkin_matches_dense(dev):
    from paper_2508_13386_amd import ms
    s, c = _setup(dev)
    B = c.ms_get_basis()
    say("basis m", B["m"], "nnz", len(B["vphi"]))
    rng = np.random.default_rng(0)
    x = s["rest"] + 0.002 * rng.standard_normal(s["rest"].shape)
    _, _, Hb = c.ms_eval(x, s["dt"])
    rp, col = c.ms_get_pattern()
    H = linops.bsr_matrix(rp, col, Hb, len(x))
    U, _ = _dense_U(s, B)
    Aref = linops.galerkin(U, H)
    A = c.ms_get_coarse_matrix(12 * B["m"])
    assert np.abs(A - Aref).max() <= 1e-11 * np.abs(Aref).max()
    c.close()


def test_two_level_apply_matches_dense(dev):
    from paper_2508_13386_amd import ms
    s, c = _setup(dev)
    B = c.ms_get_basis()
    x = s["rest"].copy()
    _, _, Hb = c.ms_eval(x, s["dt"])
    rp, col = c.ms_get_pattern()
    H = linops.bsr_matrix(rp, col, Hb, len(x))
    U, pinned = _dense_U(s, B)
    A = linops.galerkin(U, H)
    r = np.random.default_rng(1).standard_normal(x.shape)
    r[pinned] = 0.0
    Dinv = linops.block_jacobi_inverse(rp, col, Hb, len(x))
    Dinv[pinned] = 0.0
    # regularise exactly like the library: null rows of A get the largest diagonal
    d = np.diag(A).copy()
    bad = ~(d > 1e-14 * d.max())
    A[bad, bad] = d.max()
    Q = lambda v: linops.prolong(U, linops.coarse_solve(A, linops.restrict(U, v)))
    Sr = np.einsum("vij,vj->vi", Dinv, r)
    # additive: z = S r + Q r
    zref = Sr + Q(r)
    z = c.ms_apply_preconditioner(ms.PC_TWO_LEVEL_ADDITIVE, r)
    assert np.abs(z - zref).max() <= 1e-9 * np.abs(zref).max()
    r2 = np.random.default_rng(2).standard_normal(x.shape)
    r2[pinned] = 0.0
    z2 = c.ms_apply_preconditioner(ms.PC_TWO_LEVEL_ADDITIVE, r2)
    assert abs((z * r2).sum() - (z2 * r).sum()) <= 1e-10 * abs((z * r2).sum())
    assert (z * r).sum() > 0
    # smoothing then coarse correction: z = S r + Q (r - H S r)
    t = r - linops.bsr_matvec(rp, col, Hb, Sr)
    t[pinned] = 0.0
    zref = Sr + Q(t)
    z = c.ms_apply_preconditioner(ms.PC_TWO_LEVEL, r)
    assert np.abs(z - zref).max() <= 1e-9 * np.abs(zref).max()
    # symmetric V(1,1) with the l1-scaled block-Jacobi smoother L:
    # z1 = L r, z2 = z1 + Q (r - H z1), z = z2 + L (r - H z2)
    V = np.asarray(Hb, dtype=np.float64).reshape(-1, 3, 3)
    L = np.zeros((len(x), 3, 3))
    for i in range(len(x)):
        if pinned[i]:
            continue
        D, l1 = None, np.zeros(3)
        for k in range(rp[i], rp[i + 1]):
            if col[k] == i:
                D = V[k].copy()
            elif not pinned[col[k]]:
                l1 += np.abs(V[k]).sum(axis=1)
        L[i] = np.linalg.inv(D + np.diag(l1))
    Hm = lambda y: linops.bsr_matvec(rp, col, Hb, y)

    def vcycle(v):
        z1 = np.einsum("vij,vj->vi", L, v)
        t1 = v - Hm(z1)
        t1[pinned] = 0.0
        z2 = z1 + Q(t1)
        t2 = v - Hm(z2)
        t2[pinned] = 0.0
        return z2 + np.einsum("vij,vj->vi", L, t2)

    zv = c.ms_apply_preconditioner(ms.PC_TWO_LEVEL_VCYCLE, r)
    zref = vcycle(r)
    assert np.abs(zv - zref).max() <= 1e-9 * np.abs(zref).max()
    zv2 = c.ms_apply_preconditioner(ms.PC_TWO_LEVEL_VCYCLE, r2)
    assert abs((zv * r2).sum() - (zv2 * r).sum()) <= 1e-10 * abs((zv * r2).sum())
    assert (zv * r).sum() > 0
    # the plain block-Jacobi inverses are back after a V-cycle application
    zbj = c.ms_apply_preconditioner(ms.PC_BLOCK_JACOBI, r)
    assert np.abs(zbj - Sr).max() <= 1e-12 * np.abs(Sr).max()
    c.close()


@pytest.mark.parametrize("prec_name,m,path", [("fp64", 16, "direct"), ("mixed", 16, "direct"),
                                              ("fp64", 130, "gemv tail"), ("fp64", 2, "multi-chunk"),
                                              ("mixed", 2, "multi-chunk")])
def test_two_level_additive_apply_several_blocks(dev, prec_name, m, path):
    """The additive preconditioner (restriction by update-block segments, as
    in the PCG loop) on a mesh spanning several 256-vertex blocks with a
    ragged last block; mixed precision applies FP32 inverses.  The cases also
    reach the two coarse paths the benchmarked forms take: an FP64 coarse
    GEMV over more than 1280 columns (the loop after the preloaded row
    pieces; the FP64 bench form has r = 2304), and handles with more than
    1024 basis entries, whose restriction spans several chunks so that the
    GEMV sums chunk partials per handle.  The tail case runs on the plain
    cube: 170 handles on the 12^3 block with its 1e5 contrast make U^T H U
    numerically singular (condition 3e16, so the regularisation of null
    pivots, not the GEMV, would decide the comparison), while on the cube
    the condition number is about 1e6."""
    from paper_2508_13386_amd import ms
    prec = ms.PREC_MIXED if prec_name == "mixed" else ms.PREC_FP64
    s, c = _setup(dev, N=12, m=m, seed=3, scene="plain_cube" if path == "gemv tail" else "inclusion_block")
    B = c.ms_get_basis()
    per_handle = np.bincount(B["vhandle"], minlength=B["m"])
    say("n", len(s["rest"]), "basis m", B["m"], "r", 12 * B["m"], "nnz", len(B["vphi"]),
        "largest handle", int(per_handle.max()), prec_name, path)
    if path == "gemv tail":
        assert 12 * B["m"] > 1280
    elif path == "multi-chunk":
        assert per_handle.max() > 1024
    x = s["rest"] + 0.001 * np.random.default_rng(5).standard_normal(s["rest"].shape)
    _, _, Hb = c.ms_eval(x, s["dt"], prec=prec)
    rp, col = c.ms_get_pattern()
    H = linops.bsr_matrix(rp, col, Hb, len(x))
    U, pinned = _dense_U(s, B)
    A = linops.galerkin(U, H)
    d = np.diag(A).copy()
    bad = ~(d > 1e-14 * d.max())
    A[bad, bad] = d.max()
    Dinv = linops.block_jacobi_inverse(rp, col, Hb, len(x))
    Dinv[pinned] = 0.0
    tol = 1e-9 if prec == ms.PREC_FP64 else 2e-5
    zs = []
    for seed in (7, 8):
        r = np.random.default_rng(seed).standard_normal(x.shape)
        r[pinned] = 0.0
        zref = np.einsum("vij,vj->vi", Dinv, r) + linops.prolong(U, linops.coarse_solve(A, linops.restrict(U, r)))
        z = c.ms_apply_preconditioner(ms.PC_TWO_LEVEL_ADDITIVE, r, prec=prec)
        err = np.abs(z - zref).max() / np.abs(zref).max()
        say("apply", prec_name, "rel err", err)
        assert err <= tol
        zs.append((r, z))
    (r1, z1), (r2, z2) = zs
    assert abs((z1 * r2).sum() - (z2 * r1).sum()) <= (1e-10 if prec == ms.PREC_FP64 else 1e-6) * abs((z1 * r2).sum())
    c.close()


def test_coarse_coordinates_recover_affine_motion(dev):
    """q = (U^T M U)^-1 U^T M (x - x_rest) reproduces an affine displacement
    exactly away from Dirichlet influence (linear precision with POU)."""
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(6, seed=0)
    s["dirichlet"] = np.zeros(0, np.int32)
    c = ms.context_from_scene(dev, s)
    c.ms_build_basis(n_handles=8, seed=2)
    B = c.ms_get_basis()
    Aff = np.array([[0.01, 0.002, 0.0], [0.0, -0.003, 0.001], [0.004, 0.0, 0.002]])
    t = np.array([0.1, -0.2, 0.05])
    x = s["rest"] + s["rest"] @ Aff.T + t
    c.ms_set_state(x, np.zeros_like(x))
    q = c.ms_get_coarse(12 * B["m"])
    U = linops.dense_basis(s["rest"], B["origins"], B["vptr"], B["vhandle"], B["vphi"], B["m"])
    u = linops.prolong(U, q)
    assert np.abs(u - (x - s["rest"])).max() <= 1e-9
    c.close()


def test_two_level_steps_match_oracle(dev):
    from paper_2508_13386_amd import ms
    s, c = _setup(dev, N=8, m=10)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    x, v = s["x0"].copy(), s["v0"].copy()
    its_tl, its_bj = [], []
    for k in range(1, 4):
        xo, vo, _ = newton.newton_step(body, x, v, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](k))
        c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        for pc, its in ((ms.PC_TWO_LEVEL, its_tl), (ms.PC_TWO_LEVEL_ADDITIVE, []), (ms.PC_TWO_LEVEL_VCYCLE, []),
                        (ms.PC_BLOCK_JACOBI, its_bj)):
            c.ms_set_state(x, v)
            st = c.ms_step(s["dt"], preconditioner=pc)
            xg, _ = c.ms_get_state()
            err = e_rel(xg, xo, x)
            say("step", k, "pc", pc, "e_rel", err, "pcg", st["pcg_iters"], "newton", st["newton_iters"])
            assert err <= 1e-6
            its.append(st["pcg_iters"])
        x, v = xo, vo
    # the material-aware coarse space cuts the PCG work on the stiff-inclusion block
    assert sum(its_tl) <= 1.05 * sum(its_bj)  # never worse on a coarse space this small
    c.close()


@pytest.mark.parametrize("pc_name,opts", [
    ("additive", dict(coarse_move=0.2)),
    ("additive", dict(coarse_every=3)),
    ("smoothed", dict(coarse_move=0.2)),
    ("additive", dict(coarse_move=0.2, mixed_max_newton=1)),
    ("vcycle", dict(coarse_move=0.2)),
    ("additive", dict(coarse_move=0.2, pcg_eta_min=1e-4)),
])
def test_mixed_policies_match_oracle(dev, pc_name, opts):
    """Mixed precision with the FP64 endgame, Eisenstat-Walker forcing and a
    coarse operator that may lag the Hessian (additive form; the smoothed
    form rebuilds it every iteration) and the forced FP64 continuation:
    every step still lands on the oracle's minimiser."""
    from paper_2508_13386_amd import ms
    pc = {"additive": ms.PC_TWO_LEVEL_ADDITIVE, "smoothed": ms.PC_TWO_LEVEL,
          "vcycle": ms.PC_TWO_LEVEL_VCYCLE}[pc_name]
    s, c = _setup(dev, N=8, m=10)
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    x, v = s["x0"].copy(), s["v0"].copy()
    for k in range(1, 4):
        xo, vo, _ = newton.newton_step(body, x, v, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](k))
        c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        c.ms_set_state(x, v)
        st = c.ms_step(s["dt"], precision=ms.PREC_MIXED, preconditioner=pc, forcing=1, pcg_eta_max=0.1,
                       mixed_endgame_fp64=1, **opts)
        xg, _ = c.ms_get_state()
        err = e_rel(xg, xo, x)
        say("step", k, pc_name, opts, "e_rel", err, "pcg", st["pcg_iters"], "newton", st["newton_iters"],
            "refreshes", st["hessian_refreshes"], "escalations", st["precision_escalations"])
        assert err <= 1e-6
        if opts.get("mixed_max_newton") == 1:
            assert st["precision_escalations"] == (1 if st["newton_iters"] > 1 else 0)
        else:
            assert st["precision_escalations"] == 0
        x, v = xo, vo
    c.close()
