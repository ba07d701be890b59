"""Sparse material-aware basis weights for a given partitioning (CPU oracle).

Test infrastructure only.  Given the tet partitioning, computes the weights
phi_i of the linear-blend-skinning basis (Eq. LBS) the way Sec. 3.4 and
Sec. 3.5 describe them, with the readings listed in the design notes:

  * each partition i gets a local domain T_i = i and its face-adjacent
    partitions (two partitions are adjacent when a mesh face has a tet of
    each on its two sides);
  * on T_i solve the stiffness-weighted biharmonic equation K u = 0,
    K = L M^-1 L, where L is the P1 Laplacian with each tet's term weighted
    by its Young's modulus and M the lumped vertex volumes of T_i, subject to
        u = 1 at the centre vertex of i,
        u = 0 at the centre vertices of the neighbouring partitions,
        u = 0 on the internal boundary of T_i (vertices of faces that bound
              T_i but are shared by two tets of the mesh),
        u = 0 at Dirichlet vertices;
    the centre vertex of a partition is the vertex nearest its volume
    centroid among the non-Dirichlet vertices touching only that partition
    (else among all non-Dirichlet vertices touching it);
  * clip u to [0, inf);
  * with Dirichlet vertices, one extra weight u_DBC solved the same way on
    the partitions holding Dirichlet vertices plus their neighbours, u = 1 on
    the Dirichlet vertices and u = 0 at the centre vertices of the added
    neighbours and on the internal boundary (Sec. 3.5.1);
  * normalise: phi_i(v) = u_i(v) / (sum_j u_j(v) + u_DBC(v));
  * a free vertex that no clipped solution reaches gets weight 1 in the
    lowest-indexed partition among its tets (keeps the partition of unity);
  * handle origins are the partitions' volume centroids.

Optionally (rigid_contrast > 0, an option beside the paper's construction):
on every connected set of tets with E >= rigid_contrast x min E the rows of
the free vertices are replaced by their average over the set, the stiff
limit of the material-aware weights (each handle then moves a stiff
inclusion affinely).

The partitioning itself (geodesic K-means with pruning, Sec. 3.6) is taken
as an input here.

Pinned by tests/test_oracle_basis.py: the weighted Laplacian annihilates
constants and is exact on affine fields at interior vertices, the
constrained solution minimises u^T K u over admissible perturbations, and
the weights form a non-negative partition of unity that reproduces affine
fields and vanishes outside each local domain.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _grads(rest, tets):
    """Barycentric-coordinate gradients [T,4,3] and volumes [T]."""
    X = rest[tets]                                   # [T,4,3]
    Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)  # columns
    vol = np.linalg.det(Dm) / 6.0
    Dinv = np.linalg.inv(Dm)                         # rows = gradients of N1..N3
    g = np.zeros((len(tets), 4, 3))
    g[:, 1:] = Dinv
    g[:, 0] = -Dinv.sum(axis=1)
    return g, vol


def weighted_laplacian(rest, tets, weight, sel=None):
    """L_ab = sum_t w_t V_t grad N_a . grad N_b over the selected tets, in
    global vertex numbering; also the lumped volumes sum_t V_t / 4."""
    n = len(rest)
    tets = np.asarray(tets)
    if sel is not None:
        tets = tets[sel]
        weight = np.asarray(weight)[sel]
    g, vol = _grads(rest, tets)
    ke = np.einsum("t,tai,tbi->tab", np.asarray(weight) * vol, g, g)
    rows = np.repeat(tets, 4, axis=1).ravel()
    cols = np.tile(tets, (1, 4)).ravel()
    L = sp.csr_matrix((ke.ravel(), (rows, cols)), shape=(n, n))
    mv = np.zeros(n)
    np.add.at(mv, tets.ravel(), np.repeat(vol / 4.0, 4))
    return L, mv


def _faces(tets):
    f = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    owner = np.concatenate([np.arange(len(tets))] * 4)
    return np.sort(f, axis=1), owner


def constrained_biharmonic(L, mv, verts, fixed_vals):
    """Minimiser of u^T L M^-1 L u over the vertices `verts` (the support of
    L), with u fixed on the dict fixed_vals {vertex: value}."""
    verts = np.asarray(verts)
    Ll = L[verts][:, verts]
    K = (Ll.T @ sp.diags(1.0 / mv[verts]) @ Ll).tocsr()
    loc = {v: k for k, v in enumerate(verts)}
    fixed = np.zeros(len(verts), bool)
    u = np.zeros(len(verts))
    for v, val in fixed_vals.items():
        if v in loc:
            fixed[loc[v]] = True
            u[loc[v]] = val
    free = ~fixed
    if free.any():
        rhs = -K[free][:, fixed] @ u[fixed]
        u[free] = spla.spsolve(K[free][:, free].tocsc(), rhs)
    return u


def basis_weights(rest, tets, E, dbc, part, rigid_contrast=0.0):
    """Weights of every handle.  Returns dict(origins [m,3], rows: list per
    vertex of (handle, phi) sorted by handle, centre [m], nbr list)."""
    rest = np.asarray(rest, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    E = np.asarray(E, dtype=np.float64)
    part = np.asarray(part, dtype=np.int64)
    n, m = len(rest), int(part.max()) + 1
    is_dbc = np.zeros(n, bool)
    is_dbc[np.asarray(dbc, dtype=np.int64)] = True
    _, vol = _grads(rest, tets)
    # partition volume centroids
    cen = np.zeros((m, 3))
    pvol = np.bincount(part, weights=vol, minlength=m)
    tc = rest[tets].mean(axis=1)
    for d in range(3):
        cen[:, d] = np.bincount(part, weights=vol * tc[:, d], minlength=m) / pvol
    # partitions touching each vertex
    vparts = [set() for _ in range(n)]
    for t in range(len(tets)):
        for v in tets[t]:
            vparts[v].add(int(part[t]))
    # centre vertices
    centre = np.full(m, -1)
    for l in range(m):
        best, best_any, any_v = np.inf, np.inf, -1
        for v in range(n):
            if is_dbc[v] or l not in vparts[v]:
                continue
            dd = float(((rest[v] - cen[l]) ** 2).sum())
            if len(vparts[v]) == 1 and dd < best:
                best, centre[l] = dd, v
            if dd < best_any:
                best_any, any_v = dd, v
        if centre[l] < 0:
            centre[l] = any_v
    # face adjacency of partitions; mesh faces shared by two tets
    f, owner = _faces(tets)
    key = {}
    for k in range(len(f)):
        key.setdefault(tuple(f[k]), []).append(int(owner[k]))
    nbr = [set() for _ in range(m)]
    for own in key.values():
        if len(own) == 2 and part[own[0]] != part[own[1]]:
            a, b = int(part[own[0]]), int(part[own[1]])
            nbr[a].add(b)
            nbr[b].add(a)

    def solve_on(members, ones, zeros, zero_dbc):
        sel = np.isin(part, sorted(members))
        L, mv = weighted_laplacian(rest, tets, E, sel)
        verts = np.unique(tets[sel])
        fixed = {}
        # internal boundary: faces with one tet in the domain and two in the mesh
        cnt = {}
        for k in np.nonzero(np.concatenate([sel] * 4))[0]:
            cnt[tuple(f[k])] = cnt.get(tuple(f[k]), 0) + 1
        for fk, c in cnt.items():
            if c == 1 and len(key[fk]) == 2:
                for v in fk:
                    fixed[v] = 0.0
        if zero_dbc:
            for v in verts:
                if is_dbc[v]:
                    fixed[int(v)] = 0.0
        for v in zeros:
            fixed[int(v)] = 0.0
        for v in ones:
            fixed[int(v)] = 1.0
        u = constrained_biharmonic(L, mv, verts, fixed)
        return verts, np.maximum(u, 0.0)

    sols = []
    for i in range(m):
        members = {i} | nbr[i]
        sols.append(solve_on(members, [centre[i]], [centre[j] for j in sorted(nbr[i])], True))
    if is_dbc.any():
        core = set()
        for v in np.nonzero(is_dbc)[0]:
            core |= vparts[v]
        members = set(core)
        for l in core:
            members |= nbr[l]
        sols.append(solve_on(members, list(np.nonzero(is_dbc)[0]),
                             [centre[l] for l in sorted(members - core)], False))
    denom = np.zeros(n)
    for verts, u in sols:
        denom[verts] += u
    rows = [[] for _ in range(n)]
    for i in range(m):
        verts, u = sols[i]
        for v, val in zip(verts, u):
            if val > 0.0 and denom[v] > 0.0:
                rows[v].append((i, val / denom[v]))
    for v in range(n):
        if not denom[v] > 0.0 and not is_dbc[v] and vparts[v]:
            rows[v].append((min(vparts[v]), 1.0))
    if rigid_contrast > 0.0:
        # stiff limit: on each connected set of tets with E >= rigid_contrast
        # min E (connected through shared vertices) the free vertices take the
        # average of their rows
        E = np.asarray(E, dtype=np.float64)
        st = np.nonzero(E >= rigid_contrast * E.min())[0]
        import scipy.sparse as sps
        from scipy.sparse.csgraph import connected_components
        tv = np.asarray(tets)[st]
        adj = sps.coo_matrix((np.ones(3 * len(st)), (np.repeat(tv[:, 0], 3), tv[:, 1:].ravel())), shape=(n, n))
        _, comp = connected_components(adj, directed=False)
        in_stiff = np.zeros(n, bool)
        in_stiff[tv.ravel()] = True
        groups = {}
        for v in range(n):
            if in_stiff[v] and not is_dbc[v]:
                groups.setdefault(comp[v], []).append(v)
        for vs in groups.values():
            acc = {}
            for v in vs:
                for i, w in rows[v]:
                    acc[i] = acc.get(i, 0.0) + w
            avg = sorted((i, w / len(vs)) for i, w in acc.items())
            for v in vs:
                rows[v] = list(avg)
    for v in range(n):
        rows[v].sort()
    return dict(origins=cen, rows=rows, centre=centre, nbr=[sorted(s) for s in nbr],
                dbc_weight=(sols[m] if is_dbc.any() else None))
