"""Modal moment-fitting cubature for the subspace Hessian (Sec. 3.8,
Subspace Hessian Integration: modal moment fitting and its solver; Alg. 3)
-- CPU oracle.

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module; the library never does.

What the method computes
  * Each basis function u_i is evaluated per element as the mean of its
    vertex weights phi_i over the element's four vertices (the paper's
    barycentre approximation).
  * Per partition p of the basis construction (the tets labelled p), the
    functions that touch p are gathered (sorted handle ids i_1 < ... < i_k)
    and the moment conditions of degree 2 are formed: one row each for 1,
    u_i, and u_i u_j (i <= j, lexicographic).  A[alpha, e] is the product
    for element e; the target b is the volume-weighted sum over all of the
    partition's elements, i.e. b = A vol.
  * Alg. 3: start from n_init sampled elements, solve A_S w = b by
    non-negative least squares, and while ||A_S w - b|| / ||b|| > tol add
    n_add elements drawn without replacement with probability proportional
    to rho_k = (A[:, k]^T r)^2, r = A_S w - b, then solve again.
  * The cubature subspace Hessian replaces only the elastic part (Sec. 3.8
    integrates the elastic term by cubature):
        K = U^T (M + h^2 (B'' + D'')) U + h^2 sum_q (w_q / V_q) U_q^T H_q U_q
    with H_q the element's (PSD-projected) elastic Hessian, which already
    carries its volume V_q, so w_q / V_q turns it into the cubature term.

Random numbers: draws use SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014; the finaliser of
Vigna's public-domain reference) as a counter-based generator: draw j of
partition p is mix(seed + (2^32 p + j + 1) * gamma), and its top 53 bits
give a uniform double in [0, 1).

Parity status (tests/test_oracle_cubature.py)
  element_values, moment_system   pinned: brute-force loops over vertices
                                  and elements for b; with every element
                                  selected and w = V the residual is zero
  fit_partition / fit_cubature    pinned: the residual reaches the tolerance
                                  (checked by the brute-force moments),
                                  weights are non-negative, at most as many
                                  points as moment conditions, and a single
                                  constant basis function gives one point of
                                  weight equal to the partition volume (the
                                  rank-one case the paper describes)
  cubature_galerkin               pinned: every element selected with w = V
                                  reproduces U^T H U of the assembled
                                  Hessian; positive semi-definite
  splitmix64                      pinned: the published first outputs of
                                  the reference generator from state 0
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import nnls

from .fem import barrier_d2

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(state: int) -> int:
    """Output for the state after its increment (the reference finaliser)."""
    z = state & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def uniform(seed: int, counter: int) -> float:
    """Counter-based uniform double in [0, 1): draw `counter` of stream seed."""
    z = splitmix64((seed + (counter + 1) * GAMMA) & MASK64)
    return (z >> 11) * (1.0 / (1 << 53))


def tet_volumes(rest, tets):
    X = np.asarray(rest, dtype=np.float64)[np.asarray(tets)]
    D = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    return np.abs(np.linalg.det(D)) / 6.0


def element_values(tets, vptr, vhandle, vphi, m):
    """Dense [T, m]: u_i at each element = mean of phi_i over its 4 vertices."""
    tets = np.asarray(tets)
    n = len(vptr) - 1
    W = np.zeros((n, m))
    for v in range(n):
        for k in range(vptr[v], vptr[v + 1]):
            W[v, int(vhandle[k])] += vphi[k]
    return W[tets].mean(axis=1)


def moment_system(Ue_p, vol_p):
    """Rows 1, u_i, u_i u_j (i <= j) over the functions touching the
    partition (columns of Ue_p with a nonzero); returns (A, b, handles)."""
    touch = np.nonzero(np.any(Ue_p != 0.0, axis=0))[0]
    U = Ue_p[:, touch]
    rows = [np.ones(len(Ue_p))]
    rows += [U[:, a] for a in range(len(touch))]
    for a in range(len(touch)):
        for b in range(a, len(touch)):
            rows.append(U[:, a] * U[:, b])
    A = np.array(rows)
    return A, A @ vol_p, touch


def _draw(rho, chosen, count, seed, pid, counter):
    """count draws without replacement, probability proportional to rho over
    the elements not yet chosen (in element order)."""
    rho = np.where(chosen, 0.0, rho).astype(np.float64)
    for _ in range(count):
        tot = rho.sum()
        if not tot > 0.0:
            break
        u = uniform(seed, (pid << 32) + counter) * tot
        counter += 1
        c = np.cumsum(rho)
        k = int(np.searchsorted(c, u, side="right"))
        k = min(k, len(rho) - 1)
        while rho[k] == 0.0:  # never pick a zero-weight entry at a boundary
            k -= 1
        chosen[k] = True
        rho[k] = 0.0
    return counter


def fit_partition(A, b, seed, pid, n_init, n_add, tol, max_rounds):
    """Alg. 3 on one partition: returns (local element ids, weights, rel. residual)."""
    n = A.shape[1]
    chosen = np.zeros(n, dtype=bool)
    counter = _draw(np.ones(n), chosen, min(n_init, n), seed, pid, 0)
    scale = float(b[0]) / n if b[0] > 0 else 1.0  # weights in units of the mean volume
    bn = float(np.linalg.norm(b))
    for rnd in range(max_rounds + 1):
        idx = np.nonzero(chosen)[0]
        w, _ = nnls(A[:, idx], b / scale, maxiter=50 * max(1, len(idx)))
        w = w * scale
        r = A[:, idx] @ w - b
        rel = float(np.linalg.norm(r)) / bn if bn > 0 else 0.0
        if rel <= tol or chosen.all() or rnd == max_rounds:
            break
        rho = (A.T @ r) ** 2
        counter = _draw(rho, chosen, n_add, seed, pid, counter)
    keep = w > 0.0
    return idx[keep], w[keep], rel


def fit_cubature(rest, tets, part, basis, seed=0, n_init=16, n_add=16, tol=1e-9, max_rounds=64):
    """Alg. 3 on every partition.  basis = dict(m, vptr, vhandle, vphi).
    Returns (tet ids ascending, weights, {partition: rel. residual})."""
    tets = np.asarray(tets)
    part = np.asarray(part)
    vol = tet_volumes(rest, tets)
    Ue = element_values(tets, basis["vptr"], basis["vhandle"], basis["vphi"], basis["m"])
    sel, wts, res = [], [], {}
    for p in np.unique(part):
        ids = np.nonzero(part == p)[0]
        A, b, _ = moment_system(Ue[ids], vol[ids])
        loc, w, rel = fit_partition(A, b, seed, int(p), n_init, n_add, tol, max_rounds)
        sel.append(ids[loc])
        wts.append(w)
        res[int(p)] = rel
    t = np.concatenate(sel)
    w = np.concatenate(wts)
    o = np.argsort(t)
    return t[o], w[o], res


def moment_residuals(rest, tets, part, basis, cub_tets, cub_w):
    """Relative residual of the moment conditions per partition for a given
    cubature (the check applied to cubatures built elsewhere)."""
    tets = np.asarray(tets)
    part = np.asarray(part)
    vol = tet_volumes(rest, tets)
    Ue = element_values(tets, basis["vptr"], basis["vhandle"], basis["vphi"], basis["m"])
    wfull = np.zeros(len(tets))
    wfull[np.asarray(cub_tets)] = cub_w
    out = {}
    for p in np.unique(part):
        ids = np.nonzero(part == p)[0]
        A, b, _ = moment_system(Ue[ids], vol[ids])
        out[int(p)] = float(np.linalg.norm(A @ wfull[ids] - b) / np.linalg.norm(b))
    return out


def cubature_galerkin(prob, x, Us, cub_tets, cub_w, project=True):
    """K = U^T (M + h^2 (B'' + D'')) U + h^2 sum_q (w_q / V_q) U_q^T H_q U_q.
    Us is the dense basis with zero rows on Dirichlet vertices."""
    b = prob.b
    h2 = prob.alpha * prob.h * prob.h
    cub_tets = np.asarray(cub_tets)
    He = prob.element_hessians(x, project)[cub_tets]
    s = np.asarray(cub_w, dtype=np.float64) / b.vol[cub_tets]
    r = Us.shape[1]
    K = np.zeros((r, r))
    for q, t in enumerate(cub_tets):
        dof = (3 * b.tets[t][:, None] + np.arange(3)[None, :]).ravel()
        Uq = Us[dof]
        K += (h2 * s[q]) * (Uq.T @ He[q] @ Uq)
    n = b.n
    D = np.zeros((n, 3, 3))
    D += b.mass[:, None, None] * np.eye(3)[None]
    if prob.hs is not None:
        nrm = np.asarray(prob.hs["normal"], dtype=np.float64)
        d2 = barrier_d2(prob._dist(x), float(prob.hs["dhat"]))
        D += h2 * float(prob.hs["kappa"]) * d2[:, None, None] * np.outer(nrm, nrm)[None]
    if prob.fric is not None:
        D += h2 * prob.friction_blocks(x)
    for v in range(n):
        Uv = Us[3 * v:3 * v + 3]
        if np.any(Uv):
            K += Uv.T @ D[v] @ Uv
    return K
