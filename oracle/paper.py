"""The paper's three-level inexact Newton timestep (Alg. 1 and Alg. 2), FP64
CPU oracle.  Test infrastructure only.

Per Newton iteration at x, with g = grad E(x) and the PSD-projected Hessian
H (the exact Galerkin products stand in for the paper's cubature Hessian):

  1. affine level: U_a^T H U_a q_a = -U_a^T g, d_s = U_a q_a, where U_a is
     the per-object affine basis phi_a(v) (I_3 (x) [1, x_v - o]) with
     phi_a(v) = sum_i phi_i(v) (zero on Dirichlet vertices);
  2. sparse subspace level: U_s^T H U_s q_s = U_s^T r with r = -g - H d_s,
     d_s += U_s q_s (solved exactly; null rows of the Galerkin matrix get its
     largest diagonal entry);
  3. full-space refinement: a fixed number of 3x3 block-Jacobi PCG
     iterations on H_lag d_f = -g - H d_s from d_f = 0, with H_lag the
     elastic and inertia part of H at the last refresh plus the current
     barrier curvature;
  4. CCD-filtered Armijo backtracking along d = d_s + d_f (the subspace
     direction alone if d is not a descent direction), skipped below the
     round-off level of E as in the full-space oracle;
  5. stop after the update once mean_v ||d_s,v|| / h < eps.
The lagged part is refreshed at the first iteration and when the mean of
the last `window` accepted step sizes is below `threshold`, at most once
every `gap` iterations.

This is an approximation (the paper reports about 1% per-step error against
full IPC): its final states are *parity unpinned* against the exact
minimiser.  Its parts are pinned by tests/test_oracle_paper.py: Galerkin
orthogonality of both subspace levels, the refinement PCG against a direct
solve when run to n iterations, and convergence to the exact minimiser when
every level is solved to completion.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .cubature import cubature_galerkin
from .fem import Body, StepProblem, barrier_d2
from .linops import dense_basis
from .newton import LineSearchError, ccd_bound


def affine_weights(vptr, vphi, n):
    phia = np.zeros(n)
    for v in range(n):
        phia[v] = float(np.sum(vphi[vptr[v]:vptr[v + 1]]))
    return phia


def affine_basis(rest, phia, origin):
    """U_a (3n x 12): row block v holds phi_a(v) (I_3 (x) [1, x_v - o])."""
    n = len(rest)
    U = np.zeros((3 * n, 12))
    p = np.concatenate([np.ones((n, 1)), rest - origin], axis=1)  # [n,4]
    for a in range(3):
        U[a::3, 4 * a:4 * a + 4] = phia[:, None] * p
    return U


def block_jacobi_pcg(A, b, n_iter):
    """n_iter iterations of PCG from zero on A x = b (A sparse SPD, 3x3 block
    Jacobi preconditioner from A's diagonal blocks); stops early only on an
    exactly zero residual."""
    A = sp.csr_matrix(A)
    N = A.shape[0]
    nb = N // 3
    Dinv = np.zeros((nb, 3, 3))
    for i in range(nb):
        blk = A[3 * i:3 * i + 3, 3 * i:3 * i + 3].toarray()
        Dinv[i] = np.linalg.inv(blk) if np.abs(blk).max() > 0 else 0.0
    M = lambda r: np.einsum("vij,vj->vi", Dinv, r.reshape(nb, 3)).ravel()
    x = np.zeros(N)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    for _ in range(n_iter):
        if rz == 0.0:
            break
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


def subspace_direction(H, g, Ua, Us, Ks=None):
    """Alg. 2's SolveSubspaceDirection: returns (affine part, d_s).  Ks, if
    given, replaces the subspace matrix U_s^T H U_s (the cubature-integrated
    one of Sec. 3.8)."""
    qa = _solve_reg(Ua.T @ (H @ Ua), -(Ua.T @ g))
    da = Ua @ qa
    r = -g - H @ da
    qs = _solve_reg(Us.T @ (H @ Us) if Ks is None else Ks, Us.T @ r)
    return da, da + Us @ qs


def _barrier_diag(prob, x, h2):
    """Block-diagonal h^2 kappa b''(d) n n^T of the half-space barrier."""
    n = len(x)
    if prob.hs is None:
        return sp.csr_matrix((3 * n, 3 * n))
    nrm = np.asarray(prob.hs["normal"], dtype=np.float64)
    d2 = barrier_d2(prob._dist(x), float(prob.hs["dhat"]))
    blocks = h2 * float(prob.hs["kappa"]) * d2[:, None, None] * np.outer(nrm, nrm)[None]
    return sp.block_diag(list(blocks), format="csr")


def basis_matrices(body: Body, basis, pinned):
    """Dense U_s (zero on Dirichlet rows) and U_a with its origin."""
    n = body.n
    Us = dense_basis(body.rest, basis["origins"], basis["vptr"], basis["vhandle"], basis["vphi"], basis["m"])
    Us[np.repeat(pinned, 3)] = 0.0
    phia = affine_weights(basis["vptr"], basis["vphi"], n)
    phia[pinned] = 0.0
    origin = (body.mass[:, None] * body.rest).sum(axis=0) / body.mass.sum()
    return Us, affine_basis(body.rest, phia, origin)


def paper_step(body: Body, x_t, v_t, h, gravity, dbc, dbc_target, halfspace, basis, eps=1e-3, refine_iters=20,
               window=3, threshold=0.5, gap=5, max_newton=50, max_bt=30, record=None, cubature=None):
    """One timestep; basis = dict(origins, vptr, vhandle, vphi, m).  Returns
    (x, v, info).  cubature = (tets, weights) integrates the elastic part of
    the subspace matrix by cubature (Sec. 3.8) instead of exactly."""
    x_t = np.asarray(x_t, dtype=np.float64)
    prob = StepProblem(body, x_t, v_t, h, gravity, halfspace)
    n = body.n
    h2 = h * h
    x = x_t.copy()
    free = np.ones((n, 3), dtype=bool)
    if dbc is not None and len(dbc):
        x[np.asarray(dbc)] = np.asarray(dbc_target, dtype=np.float64)
        free[np.asarray(dbc)] = False
    fmask = free.ravel().astype(np.float64)
    pinned = ~free[:, 0]
    Us, Ua = basis_matrices(body, basis, pinned)
    Fm = sp.diags(fmask)
    alphas, last_refresh, refreshes = [], -10 ** 9, 0
    Hlag_base = None
    info = dict(newton=0, refreshes=0, alphas=[])
    for it in range(max_newton):
        g = prob.gradient(x).ravel() * fmask
        H = (Fm @ prob.hessian(x, project=True) @ Fm).tocsr()
        B = (Fm @ _barrier_diag(prob, x, h2) @ Fm).tocsr()
        refresh = it == 0
        if not refresh and len(alphas) >= max(1, window) and it - last_refresh >= gap:
            refresh = float(np.mean(alphas[-window:])) < threshold
        if refresh:
            Hlag_base = H - B
            last_refresh = it
            refreshes += 1
        Hlag = (Hlag_base + B).tocsr()
        # affine, then sparse subspace level
        Ks = None if cubature is None else cubature_galerkin(prob, x, Us, cubature[0], cubature[1])
        _, ds = subspace_direction(H, g, Ua, Us, Ks)
        # full-space refinement on the lagged Hessian
        rf = -g - H @ ds
        idx = np.nonzero(fmask)[0]
        df = np.zeros(3 * n)
        df[idx] = block_jacobi_pcg(Hlag[idx][:, idx], rf[idx], refine_iters)
        d = ds + df
        gd = float(g @ d)
        if not gd < 0.0:
            d = ds
            gd = float(g @ d)
        ds_mean = float(np.linalg.norm(ds.reshape(n, 3), axis=1).mean())
        alpha = 0.0
        if gd < 0.0:
            D = d.reshape(n, 3)
            alpha = ccd_bound(x, D, halfspace)
            E0 = prob.energy(x)
            k = 0
            # as in the full-space oracle: no backtracking once the predicted
            # decrease is below the round-off level of E
            if -gd > 1e-12 * prob.energy_scale(x):
                while prob.energy(x + alpha * D) > E0 + 1e-4 * alpha * gd:
                    alpha *= 0.5
                    k += 1
                    if k > max_bt:
                        raise LineSearchError("no decrease after %d halvings" % max_bt)
            x = x + alpha * D
        alphas.append(alpha)
        if record is not None:
            record.append(dict(ds_mean=ds_mean, alpha=alpha, refresh=refresh))
        if ds_mean / h < eps or gd >= 0.0:
            info.update(newton=it + 1, refreshes=refreshes, alphas=alphas)
            return x, (x - x_t) / h, info
    raise RuntimeError("paper-mode Newton did not meet its termination rule")


def _solve_reg(A, b):
    """Solve the symmetric system, giving null rows the largest diagonal."""
    A = 0.5 * (A + A.T)
    d = np.diag(A).copy()
    dmax = d.max() if d.max() > 0 else 1.0
    bad = ~(d > 1e-14 * dmax)
    A = A.copy()
    A[bad, :] = 0.0
    A[:, bad] = 0.0
    A[bad, bad] = dmax
    return np.linalg.solve(A, np.where(bad, 0.0, b))
