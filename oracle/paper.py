"""The paper's three-level inexact Newton timestep (Alg. 1 with the linear
solves of Alg. 2), FP64 CPU oracle.  Test infrastructure only.

Per Newton iteration at x, with g = grad E(x) and the PSD-projected Hessian
H (exact, or, when a cubature is given, the cubature-integrated Hessian of
Sec. 3.8 on both subspace levels; the refinement residual always takes the
exact full-space H):

  1. lag trigger (Sec. 3.7.2, Hessian lagging): the lagged elastic and
     inertia part of H is recomputed at the first iteration of the step and
     whenever the mean of the last `window` accepted step sizes is below
     `threshold`, at most once every `gap` iterations (lag_should_refresh);
  2. affine level (Alg. 2, Sec. 3.7.1): (U_a^T H U_a) q_a = -U_a^T g by PCG
     with the 12 x 12 block-Jacobi preconditioner (one block per object: the
     affine basis of one body has 12 columns), from q_a = 0 to a relative
     residual of `rtol`; d_s = U_a q_a;
  3. sparse subspace level (Alg. 2, Sec. 3.7.1): r = -g - H d_s, then
     (U_s^T H U_s) q_s = U_s^T r by PCG with one 12 x 12 Jacobi block per
     handle (the 12 DOFs of a handle), from q_s = 0 to the relative residual
     `rtol`; d_s += U_s q_s;
  4. full-space refinement (Sec. 3.7.2): a fixed number of PCG iterations
     with the diagonal (Jacobi) preconditioner on H_lag d_f = -g - H d_s from
     d_f = 0, where H_lag is the lagged part plus the current barrier
     curvature (contact terms are always recomputed); the count is 20 or 40,
     whichever is closer to the partitions' mean hop diameter
     (refine_iterations);
  5. CCD-filtered Armijo backtracking along d = d_s + d_f (Sec. 3.9; the
     subspace direction alone if d is not a descent direction), skipped
     below the round-off level of E as in the full-space oracle;
  6. stop after the update once the mean per-vertex norm of d_s divided by
     h is below eps (Alg. 1 termination, Sec. 3.9).

Readings where the paper is silent (shared with the GPU library):
  * with a cubature, the affine and sparse levels both take the cubature
    Hessian (Sec. 3.7.1: both solves use the same approximation), i.e. the
    blocks of U^T H_cub U on the stacked basis [U_s, U_a]; the refinement's
    right-hand side -g - H d_s takes the exact H, the full-space operator
    the refinement works on;
  * the signs of Alg. 2 are taken so that d is a descent direction for
    g = grad E (the printed right-hand sides U_a^T g and g - H d_s are the
    negatives of the ones solved here);
  * PCG stops when the recursive residual satisfies ||r_k|| <= rtol ||r_0||
    (2-norms; r_0 = b since every solve starts from zero), checked before
    every iteration, or after `max_iter` iterations, or when p^T A p <= 0;
  * a 12 x 12 Jacobi block is applied through its LDL^T generalised
    inverse, a pivot not above 1e-10 of its diagonal entry counting as zero
    (a handle with no free vertex has a zero block; one whose free vertices
    are coplanar has a rank-deficient one, and the right-hand side has no
    component along its null directions);
  * the hop diameter of a partition is the largest breadth-first edge-hop
    distance, over the mesh edges that join two vertices of the partition's
    tets, from the partition vertex nearest the handle origin; the mean over
    partitions is binned to 20 when it is at most 30 and to 40 otherwise
    (an exact tie goes to 20).

This is an approximation (the paper reports about 1% per-step error against
full IPC): its final states are *parity unpinned* against the exact
minimiser.  Its parts are pinned by tests/test_oracle_paper.py: the PCG stop
rule (met at the returned iterate and not one iteration earlier), one
iteration for block-diagonal systems, the direct solve when run to
completion, Galerkin orthogonality of both levels, the lag trigger on a
scripted step-size sequence worked out by hand, the hop rule against the
closed-form graph distance of the Kuhn lattice, and convergence to the
exact minimiser when every level is solved to completion.
"""
from __future__ import annotations

from collections import deque

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


# -- PCG variants ------------------------------------------------------------

def pcg(A, b, apply_M, rtol, max_iter):
    """Preconditioned conjugate gradient from x = 0 on A x = b (A symmetric,
    dense or sparse; apply_M applies the preconditioner).  Stops before an
    iteration once ||r|| <= rtol ||b||, after max_iter iterations, or when
    p^T A p <= 0.  Returns (x, iterations)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = float(np.linalg.norm(b))
    it = 0
    if bnorm == 0.0:
        return x, 0
    z = apply_M(r)
    p = z.copy()
    rz = float(r @ z)
    while it < max_iter and float(np.linalg.norm(r)) > rtol * bnorm:
        q = A @ p
        pq = float(p @ q)
        if not pq > 0.0:
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        z = apply_M(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it


def ldl_pinv(B, piv_tol=1e-10):
    """Generalised inverse of a symmetric positive semi-definite block through
    its LDL^T factorisation in natural order: a pivot not above piv_tol times
    the block's original diagonal entry counts as zero (for a PSD matrix a
    zero pivot has a zero column below it, so B = L D L^T still holds) and
    contributes nothing; the result is L^-T D^+ L^-1, which satisfies
    B X B = B."""
    B = np.asarray(B, dtype=np.float64)
    k = B.shape[0]
    L = np.eye(k)
    d = np.zeros(k)
    for j in range(k):
        dj = B[j, j] - sum(L[j, q] * L[j, q] * d[q] for q in range(j))
        if not dj > piv_tol * B[j, j]:
            continue  # zero pivot: column j of L stays e_j, d_j = 0
        d[j] = dj
        for i in range(j + 1, k):
            L[i, j] = (B[i, j] - sum(L[i, q] * L[j, q] * d[q] for q in range(j))) / dj
    Linv = np.linalg.inv(L)  # unit lower triangular
    dplus = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    return Linv.T @ (dplus[:, None] * Linv)


def block_jacobi_dense(A, bs=12):
    """Preconditioner applying the generalised inverses (ldl_pinv) of the
    bs x bs diagonal blocks of the dense matrix A."""
    A = np.asarray(A, dtype=np.float64)
    N = A.shape[0]
    nbk = N // bs
    inv = np.zeros((nbk, bs, bs))
    for k in range(nbk):
        inv[k] = ldl_pinv(A[k * bs:(k + 1) * bs, k * bs:(k + 1) * bs])
    return lambda r: np.einsum("kij,kj->ki", inv, r.reshape(nbk, bs)).ravel()


def jacobi(A):
    """Diagonal (Jacobi) preconditioner of a sparse or dense matrix."""
    d = A.diagonal() if sp.issparse(A) else np.diag(A)
    dinv = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    return lambda r: dinv * r


def block_pcg(A, b, rtol, bs=12, max_iter=100000):
    """PCG with the bs x bs block-Jacobi preconditioner to relative residual
    rtol (the affine and sparse subspace solves of Alg. 2)."""
    return pcg(A, b, block_jacobi_dense(A, bs), rtol, max_iter)


def jacobi_pcg(A, b, n_iter):
    """n_iter iterations of Jacobi-preconditioned CG from zero (the full-space
    refinement of Sec. 3.7.2); stops early only on an exactly zero residual
    or a loss of positive curvature."""
    A = sp.csr_matrix(A) if sp.issparse(A) else np.asarray(A)
    return pcg(A, b, jacobi(A), 0.0, n_iter)[0]


# -- lag trigger and refinement count -----------------------------------------

def lag_should_refresh(it, alphas, last_refresh, window=3, threshold=0.5, gap=5):
    """Hessian-lag trigger of Sec. 3.7.2 at Newton iteration it (0-based),
    given the accepted step sizes of iterations 0..it-1 and the iteration of
    the last refresh."""
    if it == 0:
        return True
    if len(alphas) < max(1, window) or it - last_refresh < gap:
        return False
    return float(np.mean(alphas[-window:])) < threshold


def partition_hop_diameters(rest, tets, part, origins):
    """Per partition: the largest edge-hop distance from the partition vertex
    nearest its handle origin to any vertex of the partition, over mesh edges
    joining two of its vertices (breadth-first search).  Partitions with no
    tet are skipped (NaN)."""
    tets = np.asarray(tets)
    part = np.asarray(part)
    n = len(rest)
    nbr = [set() for _ in range(n)]
    for t in tets:
        for a in range(4):
            for b in range(4):
                if a != b:
                    nbr[int(t[a])].add(int(t[b]))
    m = len(origins)
    out = np.full(m, np.nan)
    for l in range(m):
        verts = np.unique(tets[part == l].ravel())
        if len(verts) == 0:
            continue
        inside = set(int(v) for v in verts)
        d2 = ((rest[verts] - origins[l]) ** 2).sum(axis=1)
        start = int(verts[int(np.argmin(d2))])
        dist = {start: 0}
        q = deque([start])
        while q:
            v = q.popleft()
            for w in nbr[v]:
                if w in inside and w not in dist:
                    dist[w] = dist[v] + 1
                    q.append(w)
        out[l] = max(dist.values())
    return out


def refine_iterations(rest, tets, part, origins):
    """Refinement CG count of Sec. 3.7.2: 20 or 40, whichever is closer to the
    mean hop diameter of the partitions (20 on a tie).  Returns (count,
    mean hop diameter)."""
    d = partition_hop_diameters(rest, tets, part, origins)
    mean = float(np.nanmean(d))
    return (20 if mean <= 30.0 else 40), mean


# -- Alg. 2 --------------------------------------------------------------------

def subspace_direction(H, g, Ua, Us, K=None, rtol=1e-4, max_iter=100000):
    """Alg. 2's SolveSubspaceDirection: returns (affine part, d_s, PCG
    iterations of the affine level, of the sparse level).  Both levels use
    the same Hessian approximation (Sec. 3.7.1): the full-space H, or, when
    K is given, the cubature-integrated one of Sec. 3.8 through its subspace
    blocks K = dict(ss=U_s^T H U_s, sa=U_s^T H U_a, aa=U_a^T H U_a)."""
    Aa = Ua.T @ (H @ Ua) if K is None else K["aa"]
    qa, ia = block_pcg(Aa, -(Ua.T @ g), rtol, 12, max_iter)
    da = Ua @ qa
    if K is None:
        As, rhs = Us.T @ (H @ Us), Us.T @ (-g - H @ da)
    else:
        As, rhs = K["ss"], -(Us.T @ g) - K["sa"] @ qa
    qs, is_ = block_pcg(As, rhs, rtol, 12, max_iter)
    return da, da + Us @ qs, ia, is_


def cubature_blocks(prob, x, Us, Ua, cub_tets, cub_w):
    """The cubature-integrated Hessian's blocks on the sparse and affine
    bases (one integration over the stacked basis [U_s, U_a])."""
    rs = Us.shape[1]
    K = cubature_galerkin(prob, x, np.hstack([Us, Ua]), cub_tets, cub_w)
    return dict(ss=K[:rs, :rs], sa=K[:rs, rs:], aa=K[rs:, rs:])


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


def paper_step(body: Body, x_t, v_t, h, gravity, dbc, dbc_target, halfspace, basis, eps=1e-3, refine_iters=None,
               window=3, threshold=0.5, gap=5, max_newton=50, max_bt=30, record=None, cubature=None,
               rtol=1e-4, max_pcg=100000):
    """One timestep; basis = dict(origins, vptr, vhandle, vphi, m[, part]).
    Returns (x, v, info).  refine_iters None takes the hop rule (needs
    basis["part"]).  cubature = (tets, weights) integrates the elastic part
    of the subspace matrix by cubature (Sec. 3.8) instead of exactly."""
    x_t = np.asarray(x_t, dtype=np.float64)
    prob = StepProblem(body, x_t, v_t, h, gravity, halfspace)
    n = body.n
    h2 = h * h
    if refine_iters is None:
        refine_iters = refine_iterations(body.rest, body.tets, basis["part"], basis["origins"])[0]
    x = x_t.copy()
    free = np.ones((n, 3), dtype=bool)
    if dbc is not None and len(dbc):
        x[np.asarray(dbc)] = np.asarray(dbc_target, dtype=np.float64)
        free[np.asarray(dbc)] = False
    fmask = free.ravel().astype(np.float64)
    pinned = ~free[:, 0]
    Us, Ua = basis_matrices(body, basis, pinned)
    Fm = sp.diags(fmask)
    idx = np.nonzero(fmask)[0]
    alphas, last_refresh, refreshes = [], -10 ** 9, 0
    Hlag_base = None
    info = dict(newton=0, refreshes=0, alphas=[], affine_iters=0, subspace_iters=0, refine_iters=refine_iters)
    for it in range(max_newton):
        g = prob.gradient(x).ravel() * fmask
        H = (Fm @ prob.hessian(x, project=True) @ Fm).tocsr()
        B = (Fm @ _barrier_diag(prob, x, h2) @ Fm).tocsr()
        refresh = lag_should_refresh(it, alphas, last_refresh, window, threshold, gap)
        if refresh:
            Hlag_base = H - B
            last_refresh = it
            refreshes += 1
        Hlag = (Hlag_base + B).tocsr()
        # affine, then sparse subspace level
        K = None if cubature is None else cubature_blocks(prob, x, Us, Ua, cubature[0], cubature[1])
        _, ds, ia, is_ = subspace_direction(H, g, Ua, Us, K, rtol, max_pcg)
        info["affine_iters"] += ia
        info["subspace_iters"] += is_
        # full-space refinement on the lagged Hessian
        rf = -g - H @ ds
        df = np.zeros(3 * n)
        df[idx] = jacobi_pcg(Hlag[idx][:, idx], rf[idx], refine_iters)
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
            record.append(dict(ds_mean=ds_mean, alpha=alpha, refresh=refresh, affine_iters=ia, subspace_iters=is_))
        if ds_mean / h < eps or gd >= 0.0:
            info.update(newton=it + 1, refreshes=refreshes, alphas=alphas)
            return x, (x - x_t) / h, info
    raise RuntimeError("paper-mode Newton did not meet its termination rule")
