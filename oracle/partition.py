"""Material-aware mesh partitioning by geodesic K-means (CPU oracle).

Test infrastructure only: the tests may use this module; the library never
does.

Sec. 3.6 partitions the mesh for the basis handles: distances grow slowly
inside stiff material and quickly across material jumps (Sec. 3.6.1, 3.6.2),
and K-means under that distance places the partitions (Sec. 3.6.3).  The
readings taken here (listed in the design notes):

  * distance: shortest paths on the mesh's edge graph (the paper computes a
    heat-method geodesic; the graph metric is the reading), each edge
    costing its rest length times sqrt(w_ref / w_edge), w_edge the mean
    stiffness of the tets containing the edge, w_ref the median tet
    stiffness;
  * stiffness: Young's modulus, except that every tet touching a vertex
    shared by tets of different moduli takes jump * min(E) (the jump
    penalty of Sec. 3.6.2);
  * seeds: here the deterministic lattice seeding (the vertex nearest each
    point of a k x k x k lattice over the bounding box, k = round(m^(1/3)),
    duplicates dropped); the library's randomised kmeans++ seeding with
    pruning is not reproduced;
  * Lloyd iteration: vertices take the nearest seed (ties to the lower seed
    index), each tet the label held by most of its vertices (ties to the
    label whose vertices come nearer their seed, then to the first vertex
    in tet order), and each seed moves to the vertex of its partition
    nearest the partition's volume centroid (ties to the lower vertex id),
    until the seeds stop moving or after max_lloyd rounds;
  * labels are numbered in order of first appearance over the tets.

Parity status (tests/test_oracle_partition.py)
  geodesic distances   pinned: against Bellman-Ford relaxation written out
                       on small meshes, and Euclidean edge lengths on a
                       homogeneous material
  stiffness            pinned: jump penalty on the tets touching a material
                       interface, none elsewhere
  Voronoi labels       pinned: every vertex's seed is a nearest one by
                       brute force over all seeds
  Lloyd result         pinned: a fixed point of its own update, and every
                       partition's seed lies in it
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg


def tet_stiffness(E, tets, jump):
    """Per-tet stiffness with the jump penalty."""
    E = np.asarray(E, dtype=np.float64)
    tets = np.asarray(tets)
    n = int(tets.max()) + 1
    vmin = np.full(n, np.inf)
    vmax = np.zeros(n)
    np.minimum.at(vmin, tets.ravel(), np.repeat(E, 4))
    np.maximum.at(vmax, tets.ravel(), np.repeat(E, 4))
    mixed = vmax > vmin * (1.0 + 1e-12)
    w = E.copy()
    w[mixed[tets].any(axis=1)] = jump * E.min()
    return w


def edge_graph(rest, tets, w):
    """Symmetric sparse matrix of edge costs |x_i - x_j| sqrt(w_ref / w_edge)."""
    rest = np.asarray(rest, dtype=np.float64)
    tets = np.asarray(tets)
    n = len(rest)
    wref = float(np.sort(w)[len(w) // 2])
    pairs = [(a, b) for a in range(4) for b in range(4) if a != b]
    # tet-major order, so that each edge's stiffness sum runs over its tets in order
    i = np.stack([tets[:, a] for a, b in pairs], axis=1).ravel()
    j = np.stack([tets[:, b] for a, b in pairs], axis=1).ravel()
    ww = np.repeat(np.asarray(w, dtype=np.float64), len(pairs))
    key = i.astype(np.int64) * n + j
    uk, inv = np.unique(key, return_inverse=True)
    wsum = np.bincount(inv, weights=ww)
    cnt = np.bincount(inv)
    ei, ej = uk // n, uk % n
    L = np.sqrt(((rest[ei] - rest[ej]) ** 2).sum(axis=1))
    cost = L * np.sqrt(wref / np.maximum(wsum / cnt, 1e-300))
    return sp.csr_matrix((cost, (ei, ej)), shape=(n, n))


def voronoi(G, seeds):
    """(label [n], dist [n]): nearest seed (index into seeds) and distance."""
    D = csg.dijkstra(G, directed=True, indices=np.asarray(seeds))
    dist = D.min(axis=0)
    label = np.argmin(D, axis=0)  # first (lowest seed index) among equals
    return label, dist


def lattice_seeds(rest, m):
    rest = np.asarray(rest, dtype=np.float64)
    lo, hi = rest.min(axis=0), rest.max(axis=0)
    k = max(1, int(round(m ** (1.0 / 3.0))))
    seeds = []
    for a in range(k):
        for b in range(k):
            for e in range(k):
                p = lo + (np.array([a, b, e]) + 0.5) * (hi - lo) / k
                v = int(np.argmin(((rest - p) ** 2).sum(axis=1)))
                if v not in seeds:
                    seeds.append(v)
    return seeds


def tet_labels(tets, label, dist):
    out = np.empty(len(tets), dtype=np.int64)
    for t, tv in enumerate(np.asarray(tets)):
        best, bc, bd = -1, 0, np.inf
        for a in range(4):
            la = label[tv[a]]
            same = [b for b in range(4) if label[tv[b]] == la]
            cnt = len(same)
            dmin = min(dist[tv[b]] for b in same)
            if cnt > bc or (cnt == bc and dmin < bd):
                best, bc, bd = la, cnt, dmin
        out[t] = best
    return out


def volumes_centroids(rest, tets, vol, tl, k):
    """Partition volumes and volume-weighted vertex sums (each tet adds a
    quarter of its volume at each of its vertices, tets in order)."""
    pv = np.bincount(tl, weights=vol, minlength=k)
    cen = np.zeros((k, 3))
    xv = np.asarray(rest)[np.asarray(tets)]  # [T,4,3]
    for d in range(3):
        cen[:, d] = np.bincount(np.repeat(tl, 4), weights=(np.asarray(vol)[:, None] * 0.25 * xv[:, :, d]).ravel(),
                                minlength=k)
    return pv, cen


def lloyd(rest, tets, vol, G, seeds, max_lloyd=50):
    """(tet labels, seeds) of the Lloyd iteration from the given seeds: the
    labels of the last labelling (the seeds it used, when the budget ends
    the iteration, are the ones before the last move)."""
    seeds = list(seeds)
    tets = np.asarray(tets)
    used = list(seeds)
    for _ in range(max(1, max_lloyd)):
        label, dist = voronoi(G, seeds)
        tl = tet_labels(tets, label, dist)
        used = list(seeds)
        k = len(seeds)
        pv, cen = volumes_centroids(rest, tets, vol, tl, k)
        new = list(seeds)
        for l in range(k):
            if not pv[l] > 0:
                continue
            c = cen[l] / pv[l]
            verts = np.unique(tets[tl == l].ravel())
            verts = verts[label[verts] == l]
            d2 = ((np.asarray(rest)[verts] - c) ** 2).sum(axis=1)
            new[l] = int(verts[np.argmin(d2)])  # first minimum: lowest vertex id (verts ascending)
        if new == seeds:
            break
        seeds = new
    return tl, used


def compact(tl):
    remap = {}
    out = np.empty_like(tl)
    for t, l in enumerate(tl):
        if l not in remap:
            remap[l] = len(remap)
        out[t] = remap[l]
    return out


def partition(rest, tets, E, vol, m, jump=0.25, max_lloyd=50):
    """Lattice-seeded geodesic K-means: compact tet labels [T]."""
    w = tet_stiffness(E, tets, jump)
    G = edge_graph(rest, tets, w)
    tl, _ = lloyd(rest, tets, vol, G, lattice_seeds(rest, m), max_lloyd)
    return compact(tl)
