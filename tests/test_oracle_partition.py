"""Pins of the geodesic K-means partitioning oracle (oracle/partition.py)
and the library's host partitioning against it (lattice seeding, where no
random draw is involved)."""
import math

import numpy as np
import pytest

import scenes
from oracle import fem
from oracle import partition as pt


def _hetero(N, seed):
    rest, tets, _, _ = scenes.kuhn_cube(N)
    rng = np.random.default_rng(seed)
    E = np.exp(rng.uniform(math.log(1e5), math.log(1e8), size=len(tets)))
    return rest, tets, E


def test_geodesic_distances_against_bellman_ford():
    rest, tets, E = _hetero(2, 0)
    G = pt.edge_graph(rest, tets, pt.tet_stiffness(E, tets, 0.25)).tocoo()
    n = len(rest)
    for s in (0, 13, n - 1):
        _, dist = pt.voronoi(G.tocsr(), [s])
        d = np.full(n, np.inf)
        d[s] = 0.0
        for _ in range(n):  # relax every edge n times
            for i, j, c in zip(G.row, G.col, G.data):
                if d[i] + c < d[j]:
                    d[j] = d[i] + c
        assert np.allclose(dist, d, rtol=1e-14, atol=0)


def test_homogeneous_costs_are_edge_lengths():
    rest, tets, _, _ = scenes.kuhn_cube(3)
    E = np.full(len(tets), 3e6)
    G = pt.edge_graph(rest, tets, pt.tet_stiffness(E, tets, 0.25)).tocoo()
    L = np.sqrt(((rest[G.row] - rest[G.col]) ** 2).sum(axis=1))
    assert np.allclose(G.data, L, rtol=1e-15, atol=0)
    # every mesh edge appears in both directions with the same cost, no self loops
    Gs = G.tocsr()
    assert abs(Gs - Gs.T).max() == 0.0 and np.all(G.row != G.col)


def test_jump_penalty_on_interface_tets_only():
    rest, tets, _, _ = scenes.kuhn_cube(4)
    bary = rest[tets].mean(axis=1)
    E = np.where(bary[:, 0] < 0.5, 1e5, 1e9)
    w = pt.tet_stiffness(E, tets, 0.25)
    n = len(rest)
    mixed = np.zeros(n, bool)
    for v in range(n):
        es = E[(tets == v).any(axis=1)]
        mixed[v] = es.min() != es.max()
    touch = mixed[tets].any(axis=1)
    assert touch.any() and (~touch).any()
    assert np.all(w[touch] == 0.25 * 1e5)
    assert np.array_equal(w[~touch], E[~touch])


def test_voronoi_labels_are_nearest_seeds():
    rest, tets, E = _hetero(4, 1)
    G = pt.edge_graph(rest, tets, pt.tet_stiffness(E, tets, 0.25))
    seeds = [0, 30, 77, 101]
    label, dist = pt.voronoi(G, seeds)
    import scipy.sparse.csgraph as csg
    D = np.stack([csg.dijkstra(G, indices=s) for s in seeds])
    assert np.allclose(dist, D.min(axis=0), rtol=1e-15, atol=0)
    assert np.all(D[label, np.arange(len(rest))] == D.min(axis=0))


def test_lloyd_result_is_a_fixed_point():
    rest, tets, E = _hetero(5, 2)
    vol = fem.Body(rest, tets, E, np.full(len(tets), 0.4), np.full(len(tets), 1e3)).vol
    G = pt.edge_graph(rest, tets, pt.tet_stiffness(E, tets, 0.25))
    seeds0 = pt.lattice_seeds(rest, 8)
    assert len(seeds0) == 8
    tl, seeds = pt.lloyd(rest, tets, vol, G, seeds0, max_lloyd=100)
    tl2, seeds2 = pt.lloyd(rest, tets, vol, G, seeds, max_lloyd=1)
    assert seeds2 == seeds and np.array_equal(tl, tl2)
    label, _ = pt.voronoi(G, seeds)
    for l, s in enumerate(seeds):
        assert label[s] == l and (tl == l).any()


@pytest.mark.parametrize("case", ["hetero6", "block8"])
def test_library_partition_matches_oracle(case):
    from paper_2508_13386_amd import ms
    if case == "hetero6":
        rest, tets, E = _hetero(6, 3)
        m = 8
    else:
        s = scenes.inclusion_block(8, seed=0)
        rest, tets, E = s["rest"], s["tets"], s["E"]
        m = 27
    vol = fem.Body(rest, tets, E, np.full(len(tets), 0.4), np.full(len(tets), 1e3)).vol
    lib = ms.ms_basis_compute(rest, tets, E, n_handles=m, lattice_seeding=1, jump_penalty=0.25, max_lloyd=50)
    orc = pt.partition(rest, tets, E, vol, m, jump=0.25, max_lloyd=50)
    assert lib["m"] == orc.max() + 1
    assert np.array_equal(lib["part"], orc)
