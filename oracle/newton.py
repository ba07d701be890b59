"""Full-space Newton timestep solve with a sparse direct solver (FP64 oracle).

Test infrastructure only.  Computes x^{t+1} = argmin E(x) of one implicit
Euler step (Sec. 3.1, Eq. IP and the Newton step H d = -g), which is the
plain definition of what the GPU's Newton-PCG path reaches: the minimiser
does not depend on the linear solver, its preconditioner, the PSD projection
or the precision of the Hessian.

Steps, in the paper's order (Sec. 3.1 and the line-search paragraph of
Sec. 3.9):
  1. x~ = x^t + h v^t; x <- x^t; prescribed (Dirichlet) vertices are set to
     their targets and their DOFs eliminated.
  2. Newton iteration: g = grad E(x), H = hess E(x) (PSD-projected elastic
     blocks), solve H_ff d_f = -g_f with SuperLU (scipy.sparse.linalg.splu).
  3. Filtered line search: the step is first truncated so that no vertex
     reaches the half-space (point-plane time of impact, 0.9 safety factor)
     and, with self-contact, so that additive CCD certifies every surface
     pair along it (Sec. 4), then backtracked by halving until the Armijo condition
     E(x + a d) <= E(x) + 1e-4 a g.d holds.  When the predicted decrease
     -g.d is below the round-off level of E (1e-12 of the sum of the absolute
     energy parts) the truncated step is taken as is.
  3b. Once ||d||_inf < 1e-6 L_bbox the exact (unprojected) Hessian is used,
     falling back to the projected one if it yields no descent direction.
  4. Stop when a full step has ||d||_inf <= 1e-12 L_bbox, or when, in the
     endgame (||d||_inf below 1e-6 L_bbox), ||d||_inf has not decreased for
     3 iterations (the round-off floor); at most 100 iterations.
  5. v^{t+1} = (x^{t+1} - x^t) / h.
A dense variant (numpy.linalg.solve) serves tiny meshes.

Pinned by tests/test_oracle_newton.py: rest state, free fall, momentum
conservation, energy decrease, dense vs sparse, small-strain limit.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fem import Body, StepProblem


class LineSearchError(RuntimeError):
    pass


def ccd_bound(x, d, halfspace, safety=0.9):
    """Largest step in [0,1] that keeps every vertex strictly above the plane:
    min over approaching vertices of safety * d_v / (-n . d_v)."""
    if halfspace is None:
        return 1.0
    n = np.asarray(halfspace["normal"], dtype=np.float64)
    dist = x @ n - float(halfspace["offset"])
    approach = -(d @ n)
    m = approach > 0
    if not m.any():
        return 1.0
    return float(min(1.0, safety * np.min(dist[m] / approach[m])))


def newton_step(body: Body, x_t, v_t, h, gravity, dbc=None, dbc_target=None, halfspace=None,
                dense=False, max_iter=100, tol=1e-12, project=True, record=None, prev=None, x_start=None,
                selfcontact=None):
    """One timestep; prev = (x^{t-1}, v^{t-1}) selects BDF2, else implicit
    Euler.  x_start (default x^t) is the first Newton iterate: the minimiser
    does not depend on it as long as it lies in the same basin, so a start
    near the answer only saves iterations.  selfcontact = dict(dhat, kappa)
    adds the IPC self-contact barrier of the body's surface; every step is
    then also truncated by the additive-CCD bound of the surface pairs."""
    x_t = np.asarray(x_t, dtype=np.float64)
    prob = StepProblem(body, x_t, v_t, h, gravity, halfspace, prev, selfcontact)
    x = (x_t if x_start is None else np.asarray(x_start, dtype=np.float64)).copy()
    n = body.n
    free = np.ones((n, 3), dtype=bool)
    if dbc is not None and len(dbc):
        x[np.asarray(dbc)] = np.asarray(dbc_target, dtype=np.float64)
        free[np.asarray(dbc)] = False
    free = free.ravel()
    L = float(np.linalg.norm(body.rest.max(axis=0) - body.rest.min(axis=0)))
    best = np.inf
    stall = 0
    its = 0
    for it in range(max_iter):
        g = prob.gradient(x).ravel()
        # PSD-projected Hessian while far from the minimiser; the exact Hessian
        # (positive definite at a stable minimiser) once the steps are small,
        # which restores Newton's quadratic convergence.
        exact = project and best < 1e-6 * L
        H = prob.hessian(x, project=project and not exact)
        Hff = H[free][:, free]
        rhs = -g[free]
        if dense:
            df = np.linalg.solve(Hff.toarray(), rhs)
        else:
            df = spla.splu(Hff.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                           options=dict(SymmetricMode=True)).solve(rhs)
        d = np.zeros(3 * n)
        d[free] = df
        d = d.reshape(n, 3)
        E0 = prob.energy(x)
        gd = float(g @ d.ravel())
        if exact and gd >= 0.0:  # not a descent direction: fall back to the projection
            best = np.inf
            continue
        alpha = ccd_bound(x, d, halfspace)
        if prob.sc is not None:
            from . import selfcontact as scm
            alpha = min(alpha, scm.ccd_bound(x, d, prob.sc["surf"]))
        if -gd > 1e-12 * prob.energy_scale(x):
            k = 0
            while prob.energy(x + alpha * d) > E0 + 1e-4 * alpha * gd:
                alpha *= 0.5
                k += 1
                if k > 30:
                    raise LineSearchError("no decrease after 30 halvings")
        x = x + alpha * d
        its = it + 1
        dinf = float(np.abs(d).max()) if d.size else 0.0
        if record is not None:
            record.append(dict(E=E0, alpha=alpha, dinf=dinf, gd=gd))
        if alpha == 1.0 and dinf <= tol * L:
            break
        if dinf < best:
            best, stall = dinf, 0
        elif best < 1e-6 * L:
            # stagnation counts only at the round-off floor of the endgame
            # (far from the minimiser backtracking makes ||d|| non-monotone)
            stall += 1
            if stall >= 3:
                break
    if prev is None:
        v = (x - x_t) / h
    else:
        v = (3.0 * x - 4.0 * x_t + np.asarray(prev[0], dtype=np.float64)) / (2.0 * h)
    return x, v, its


def simulate(scene, steps=None, dense=False, record=None):
    """Run `steps` implicit Euler steps of a scene dict from `scenes`."""
    body = Body(scene["rest"], scene["tets"], scene["E"], scene["nu"], scene["rho"])
    x = np.array(scene["x0"], dtype=np.float64)
    v = np.array(scene["v0"], dtype=np.float64)
    steps = scene["steps"] if steps is None else steps
    traj = []
    for k in range(1, steps + 1):
        x, v, its = newton_step(body, x, v, scene["dt"], scene["gravity"], scene["dirichlet"],
                                scene["dbc_targets"](k), scene["halfspace"], dense=dense)
        traj.append((x.copy(), v.copy(), its))
    return traj
