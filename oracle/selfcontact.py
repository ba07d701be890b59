"""IPC self-contact between surface primitives of a tet mesh -- CPU oracle.

Test infrastructure only: the tests may use this module; the library never
does.

The paper models contact with IPC barriers and filters every search
direction with continuous collision detection (Sec. 3.9, line search;
Sec. 4); for self-contact the constraint set is IPC's: every
point-triangle (PT) pair of a surface vertex and a surface triangle not
incident to it, and every edge-edge (EE) pair of surface edges that share
no vertex, whose unsigned distance is below d_hat.

  * Surface: the triangles of the tet mesh that belong to one tet only,
    their edges and vertices.
  * Distances: PT is the distance from the point to the closed triangle
    (the plane distance when the projection is inside, else the nearest of
    the three edges as segments); EE is the distance between the closed
    segments (the line distance when both closest parameters are interior,
    else the nearest endpoint-to-segment distance).
  * Energy: kappa sum_PT b(d) + kappa sum_EE m(c) b(d), with b the same log
    barrier as the half-space contact (in the unsigned distance d), and m
    IPC's mollifier of nearly parallel edges: c = |(a1 - a0) x (b1 - b0)|^2,
    eps_x = 1e-3 |A1 - A0|^2 |B1 - B0|^2 at rest, m = (2 - c / eps_x) c / eps_x
    for c < eps_x, else 1.
  * Gradient and Hessian of each pair's term as a function of its 12
    coordinates come from PyTorch's FP64 automatic differentiation of the
    expressions above; each 12x12 pair Hessian is projected to PSD (the
    eigen-clamp used for the elastic Hessians) before assembly.
  * Time of impact: for motion x(t) = x + t p, t in [0, 1], the first time
    the four points are coplanar (roots of the cubic triple product) with
    the point inside the triangle (PT) or the two segments crossing (EE).
  * Additive CCD, the conservative filter the paper uses (Sec. 4), as its
    authors publish it, with zero thickness.

Parity status (tests/test_oracle_selfcontact.py)
  surface                      pinned: counts and the Euler characteristic
                               of a closed cube surface
  pt_dist2, ee_dist2           pinned: closed forms per region and brute
                               force over the parameter domains
  pair energy / derivatives    pinned: central finite differences, rigid
                               invariance, mollifier closed form and C1 at
                               eps_x, zero beyond d_hat
  toi                          pinned: analytic impacts and dense sampling
                               of the distance along the motion
  accd                         pinned: never later than toi, the pair still
                               separated at the returned time, a hit
                               whenever toi finds one, translations of the
                               whole pair ignored
  candidate_pairs              pinned: the box filter loses no pair closer
                               than d_hat (equal to the brute-force set)
  ccd_bound                    pinned: never beyond the first impact of any
                               pair along the motion (dense sampling)
  in the Newton step           pinned (tests/test_oracle_newton.py): the
                               assembled gradient and Hessian against central
                               differences of the step energy, momentum
                               conservation in a collision of two free
                               bodies, separation kept along the steps
"""
from __future__ import annotations

import numpy as np
import torch

from .fem import project_psd

torch_f64 = torch.float64


# ----------------------------------------------------------------------------
# Surface of a tet mesh
# ----------------------------------------------------------------------------
def surface(tets):
    """(triangles [F,3] in ascending vertex order, edges [E,2], vertices [V])."""
    tets = np.asarray(tets)
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    faces = np.sort(faces, axis=1)
    u, cnt = np.unique(faces, axis=0, return_counts=True)
    tris = u[cnt == 1]
    e = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [0, 2]]]), axis=1)
    edges = np.unique(e, axis=0)
    verts = np.unique(tris)
    return tris, edges, verts


# ----------------------------------------------------------------------------
# Distances (torch, so that the same expressions give exact derivatives)
# ----------------------------------------------------------------------------
def _point_segment_d2(p, a, b):
    ab = b - a
    t = torch.clamp(torch.dot(p - a, ab) / torch.dot(ab, ab), 0.0, 1.0)
    c = a + t * ab
    return torch.dot(p - c, p - c)


def pt_dist2(x12):
    """Squared distance from point x12[0:3] to triangle x12[3:12]."""
    p, t0, t1, t2 = x12[0:3], x12[3:6], x12[6:9], x12[9:12]
    e0, e1 = t1 - t0, t2 - t0
    n = torch.linalg.cross(e0, e1)
    # barycentric coordinates of the projection of p
    w = p - t0
    d00, d01, d11 = torch.dot(e0, e0), torch.dot(e0, e1), torch.dot(e1, e1)
    d20, d21 = torch.dot(w, e0), torch.dot(w, e1)
    den = d00 * d11 - d01 * d01
    v = (d11 * d20 - d01 * d21) / den
    u = (d00 * d21 - d01 * d20) / den
    if v >= 0 and u >= 0 and u + v <= 1:
        h = torch.dot(w, n)
        return h * h / torch.dot(n, n)
    cands = [_point_segment_d2(p, t0, t1), _point_segment_d2(p, t1, t2), _point_segment_d2(p, t0, t2)]
    k = int(torch.argmin(torch.stack([c.detach() for c in cands])))
    return cands[k]


def ee_dist2(x12):
    """Squared distance between segments x12[0:6] and x12[6:12]."""
    a0, a1, b0, b1 = x12[0:3], x12[3:6], x12[6:9], x12[9:12]
    u, v, w = a1 - a0, b1 - b0, a0 - b0
    uu, uv, vv, uw, vw = torch.dot(u, u), torch.dot(u, v), torch.dot(v, v), torch.dot(u, w), torch.dot(v, w)
    den = uu * vv - uv * uv
    if den > 1e-12 * uu * vv:
        s = (uv * vw - vv * uw) / den
        t = (uu * vw - uv * uw) / den
        if 0 <= s <= 1 and 0 <= t <= 1:
            n = torch.linalg.cross(u, v)
            h = torch.dot(w, n)
            return h * h / torch.dot(n, n)
    cands = [_point_segment_d2(a0, b0, b1), _point_segment_d2(a1, b0, b1), _point_segment_d2(b0, a0, a1),
             _point_segment_d2(b1, a0, a1)]
    k = int(torch.argmin(torch.stack([c.detach() for c in cands])))
    return cands[k]


def mollifier(c, eps_x):
    if c < eps_x:
        r = c / eps_x
        return (2.0 - r) * r
    return torch.ones((), dtype=torch_f64)


def _barrier(d, dhat):
    return -((d - dhat) ** 2) * torch.log(d / dhat)


def pair_energy(kind, x12, dhat, eps_x=None):
    """kappa-free energy of one pair (0 beyond d_hat)."""
    d2 = pt_dist2(x12) if kind == "pt" else ee_dist2(x12)
    if not d2 < dhat * dhat:
        return torch.zeros((), dtype=torch_f64)
    e = _barrier(torch.sqrt(d2), dhat)
    if kind == "ee":
        c = torch.linalg.cross(x12[3:6] - x12[0:3], x12[9:12] - x12[6:9])
        e = mollifier(torch.dot(c, c), eps_x) * e
    return e


def pair_derivatives(kind, x12, dhat, eps_x=None, project=True, hessian=True):
    """(energy, gradient [12], Hessian [12,12] or None) of one pair."""
    x = torch.tensor(np.asarray(x12, dtype=np.float64), dtype=torch_f64)
    f = lambda y: pair_energy(kind, y, dhat, eps_x)
    e = float(f(x))
    g = torch.autograd.functional.jacobian(f, x).numpy()
    if not hessian:
        return e, g, None
    H = torch.autograd.functional.hessian(f, x).numpy()
    H = 0.5 * (H + H.T)
    if project:
        H = project_psd(H[None])[0]
        H = 0.5 * (H + H.T)
    return e, g, H


# ----------------------------------------------------------------------------
# Constraint set and assembled energy / gradient / Hessian
# ----------------------------------------------------------------------------
def eps_x_rest(rest, a0, a1, b0, b1):
    return 1e-3 * float(np.sum((rest[a1] - rest[a0]) ** 2)) * float(np.sum((rest[b1] - rest[b0]) ** 2))


def active_pairs(x, surf, dhat):
    """Every PT and EE pair with distance < d_hat (brute force)."""
    tris, edges, verts = surf
    x = np.asarray(x, dtype=np.float64)
    pts, ees = [], []
    for v in verts:
        for f in tris:
            if v in f:
                continue
            x12 = torch.tensor(np.concatenate([x[v], x[f[0]], x[f[1]], x[f[2]]]), dtype=torch_f64)
            if float(pt_dist2(x12)) < dhat * dhat:
                pts.append((int(v), int(f[0]), int(f[1]), int(f[2])))
    for i in range(len(edges)):
        for j in range(i + 1, len(edges)):
            a, b = edges[i], edges[j]
            if len({a[0], a[1], b[0], b[1]}) < 4:
                continue
            x12 = torch.tensor(np.concatenate([x[a[0]], x[a[1]], x[b[0]], x[b[1]]]), dtype=torch_f64)
            if float(ee_dist2(x12)) < dhat * dhat:
                ees.append((int(a[0]), int(a[1]), int(b[0]), int(b[1])))
    return pts, ees


def candidate_pairs(x, surf, pad, x2=None):
    """PT and EE pairs (incident ones excluded) whose axis-aligned boxes come
    within `pad` of each other: a superset of every pair closer than pad
    (a pair's distance is never below the gap between its boxes).
    With x2 the boxes span both positions (the motion x -> x2 is linear, so
    every pair that can meet on the way is kept).  Returns (pts, ees) as
    vertex quadruples in the order of active_pairs."""
    tris, edges, verts = surf
    x = np.asarray(x, dtype=np.float64)
    lo, hi = x.copy(), x.copy()
    if x2 is not None:
        x2 = np.asarray(x2, dtype=np.float64)
        lo, hi = np.minimum(x, x2), np.maximum(x, x2)

    def boxes(idx):
        return lo[idx].min(axis=1), hi[idx].max(axis=1)

    def near(alo, ahi, blo, bhi):
        gap = np.maximum(0.0, np.maximum(alo[:, None, :] - bhi[None, :, :], blo[None, :, :] - ahi[:, None, :]))
        return np.sqrt((gap * gap).sum(axis=2)) <= pad

    pts, ees = [], []
    vlo, vhi = lo[verts], hi[verts]
    tlo, thi = boxes(np.asarray(tris))
    for a, b in zip(*np.nonzero(near(vlo, vhi, tlo, thi))):
        v, f = int(verts[a]), tris[b]
        if v not in f:
            pts.append((v, int(f[0]), int(f[1]), int(f[2])))
    elo, ehi = boxes(np.asarray(edges))
    m = near(elo, ehi, elo, ehi)
    for i, j in zip(*np.nonzero(np.triu(m, 1))):
        a, b = edges[i], edges[j]
        if len({a[0], a[1], b[0], b[1]}) == 4:
            ees.append((int(a[0]), int(a[1]), int(b[0]), int(b[1])))
    return pts, ees


def active_pairs_filtered(x, surf, dhat):
    """active_pairs restricted to the box-filtered candidates (same result:
    a pair closer than d_hat always passes the filter)."""
    x = np.asarray(x, dtype=np.float64)
    cpt, cee = candidate_pairs(x, surf, dhat)
    pts = [q for q in cpt if float(pt_dist2(torch.tensor(x[list(q)].ravel(), dtype=torch_f64))) < dhat * dhat]
    ees = [q for q in cee if float(ee_dist2(torch.tensor(x[list(q)].ravel(), dtype=torch_f64))) < dhat * dhat]
    return pts, ees


def ccd_bound(x, d, surf, s=0.1):
    """Largest step in [0, 1] along x + t d that additive CCD certifies for
    every pair of the surface: the minimum over the pairs whose swept boxes
    meet of accd's time (pairs that cannot meet before t = 1 do not bound)."""
    x = np.asarray(x, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    cpt, cee = candidate_pairs(x, surf, 0.0, x + d)
    t = 1.0
    for kind, lst in (("pt", cpt), ("ee", cee)):
        for q in lst:
            idx = list(q)
            hit, tq = accd(kind, x[idx].ravel(), d[idx].ravel(), s=s, t_max=1.0)
            if hit:
                t = min(t, tq)
    return t


def pairs_energy(x, rest, pairs, dhat):
    """kappa-free energy summed over the given pairs (pts, ees)."""
    x = np.asarray(x, dtype=np.float64)
    E = 0.0
    for kind, lst in (("pt", pairs[0]), ("ee", pairs[1])):
        for q in lst:
            eps = eps_x_rest(rest, *q) if kind == "ee" else None
            E += float(pair_energy(kind, torch.tensor(x[list(q)].ravel(), dtype=torch_f64), dhat, eps))
    return E


def contact_terms_sparse(x, rest, pairs, dhat, kappa, project=True, hessian=True):
    """kappa-scaled energy, gradient [n,3] and sparse Hessian (CSR,
    3n x 3n; None without `hessian`) over the given pairs (pts, ees):
    contact_terms without the dense matrix."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    E = 0.0
    g = np.zeros(3 * n)
    rows, cols, vals = [], [], []
    for kind, lst in (("pt", pairs[0]), ("ee", pairs[1])):
        for q in lst:
            eps = eps_x_rest(rest, *q) if kind == "ee" else None
            x12 = np.concatenate([x[k] for k in q])
            e, gp, Hp = pair_derivatives(kind, x12, dhat, eps, project, hessian)
            dof = (3 * np.asarray(q)[:, None] + np.arange(3)[None, :]).ravel()
            E += kappa * e
            g[dof] += kappa * gp
            if not hessian:
                continue
            rows.append(np.repeat(dof, 12))
            cols.append(np.tile(dof, 12))
            vals.append(kappa * Hp.ravel())
    import scipy.sparse as sp
    if not hessian:
        return E, g.reshape(n, 3), None
    if rows:
        H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(3 * n, 3 * n)).tocsr()
    else:
        H = sp.csr_matrix((3 * n, 3 * n))
    return E, g.reshape(n, 3), H


def contact_terms(x, rest, pairs, dhat, kappa, project=True):
    """kappa-scaled energy, gradient [n,3] and dense Hessian [3n,3n] over the
    given pairs (pts, ees)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    E = 0.0
    g = np.zeros(3 * n)
    H = np.zeros((3 * n, 3 * n))
    for kind, lst in (("pt", pairs[0]), ("ee", pairs[1])):
        for q in lst:
            eps = eps_x_rest(rest, *q) if kind == "ee" else None
            x12 = np.concatenate([x[k] for k in q])
            e, gp, Hp = pair_derivatives(kind, x12, dhat, eps, project)
            dof = (3 * np.asarray(q)[:, None] + np.arange(3)[None, :]).ravel()
            E += kappa * e
            g[dof] += kappa * gp
            H[np.ix_(dof, dof)] += kappa * Hp
    return E, g.reshape(n, 3), H


# ----------------------------------------------------------------------------
# Time of impact under linear motion
# ----------------------------------------------------------------------------
def _cubic_roots(f):
    """Real roots in [0, 1] of the cubic through f(0), f(1/3), f(2/3), f(1)."""
    ts = np.array([0.0, 1.0 / 3.0, 2.0 / 3.0, 1.0])
    c = np.polyfit(ts, [f(t) for t in ts], 3)
    if np.all(np.abs(c) <= 1e-300):
        return []
    r = np.roots(c)
    r = np.real(r[np.abs(np.imag(r)) <= 1e-9 * (1.0 + np.abs(r))])
    return sorted(t for t in r if -1e-12 <= t <= 1.0 + 1e-12)


def toi(kind, x12, p12, tol=1e-9):
    """First t in [0, 1] at which the pair touches (None if it does not)."""
    x12 = np.asarray(x12, dtype=np.float64)
    p12 = np.asarray(p12, dtype=np.float64)

    def pos(t):
        return (x12 + t * p12).reshape(4, 3)

    def triple(t):
        q = pos(t)
        return float(np.dot(q[1] - q[0], np.cross(q[2] - q[0], q[3] - q[0])))

    dist = pt_dist2 if kind == "pt" else ee_dist2
    scale = max(float(np.abs(x12).max()), float(np.abs(x12 + p12).max()), 1.0)
    for t in _cubic_roots(triple):
        t = min(max(t, 0.0), 1.0)
        d2 = float(dist(torch.tensor(pos(t).ravel(), dtype=torch_f64)))
        if d2 <= (tol * scale) ** 2:
            return t
    return None


# ----------------------------------------------------------------------------
# Additive CCD (Li et al., "Codimensional Incremental Potential Contact",
# 2021): a conservative time of impact from distance evaluations only
# ----------------------------------------------------------------------------
def accd_margin(kind, x12, p12, s=0.1, t_max=1.0, max_iter=100000):
    """The smallest relative margin by which accd's run clears one of its
    decisions (the gap test |d - s d_0| / (s d_0) and the end test
    |t - t_max| / t_max, over its iterations): a run whose margin is at
    round-off level can end differently under another rounding order."""
    x = np.asarray(x12, dtype=np.float64).reshape(4, 3).copy()
    p = np.asarray(p12, dtype=np.float64).reshape(4, 3).copy()
    p = p - p.mean(axis=0)
    nrm = np.sqrt((p * p).sum(axis=1))
    lp = nrm[0] + nrm[1:].max() if kind == "pt" else max(nrm[0], nrm[1]) + max(nrm[2], nrm[3])
    if lp == 0.0:
        return np.inf
    dist = pt_dist2 if kind == "pt" else ee_dist2
    d = float(np.sqrt(float(dist(torch.tensor(x.ravel(), dtype=torch_f64)))))
    g = s * d
    t, tl, margin = 0.0, (1.0 - s) * d / lp, np.inf
    for _ in range(max_iter):
        x = x + tl * p
        d = float(np.sqrt(float(dist(torch.tensor(x.ravel(), dtype=torch_f64)))))
        if t > 0.0:
            margin = min(margin, abs(d - g) / g)
        if t > 0.0 and d < g:
            return margin
        t += tl
        margin = min(margin, abs(t - t_max) / t_max)
        if t > t_max:
            return margin
        tl = 0.9 * d / lp
    return margin


def accd(kind, x12, p12, s=0.1, t_max=1.0, max_iter=100000):
    """(hit, t): advance along x + t p in steps that cannot close more than
    90% of the current gap (the first step (1 - s) of it), given the bound
    l_p on the relative speed of the pair after removing the mean
    displacement; stop once the gap falls below s times the initial one
    (hit, t the last time before that step) or t passes t_max (no hit)."""
    x = np.asarray(x12, dtype=np.float64).reshape(4, 3).copy()
    p = np.asarray(p12, dtype=np.float64).reshape(4, 3).copy()
    p = p - p.mean(axis=0)
    nrm = np.sqrt((p * p).sum(axis=1))
    lp = nrm[0] + nrm[1:].max() if kind == "pt" else max(nrm[0], nrm[1]) + max(nrm[2], nrm[3])
    if lp == 0.0:
        return False, t_max
    dist = pt_dist2 if kind == "pt" else ee_dist2
    d = float(np.sqrt(float(dist(torch.tensor(x.ravel(), dtype=torch_f64)))))
    g = s * d
    t = 0.0
    tl = (1.0 - s) * d / lp
    for _ in range(max_iter):
        x = x + tl * p
        d = float(np.sqrt(float(dist(torch.tensor(x.ravel(), dtype=torch_f64)))))
        if t > 0.0 and d < g:
            return True, t
        t += tl
        if t > t_max:
            return False, t_max
        tl = 0.9 * d / lp
    return True, t
