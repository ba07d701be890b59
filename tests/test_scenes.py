"""Generators: sizes of the paper-shaped workloads, orientation, volume."""
import numpy as np
import pytest

import scenes


def _edges(tets, n):
    a = tets[:, [0, 0, 0, 1, 1, 2]].ravel().astype(np.int64)
    b = tets[:, [1, 2, 3, 2, 3, 3]].ravel().astype(np.int64)
    return np.unique(np.minimum(a, b) * n + np.maximum(a, b))


def _signed_vol(rest, tets):
    X = rest[tets]
    return np.einsum("ti,ti->t", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0])) / 6


@pytest.mark.parametrize("N,n,T,nnzb", [(8, 729, 3072, 9097), (32, 35937, 196608, 513313)])
def test_kuhn_counts(N, n, T, nnzb):
    rest, tets, _, _ = scenes.kuhn_cube(N)
    assert len(rest) == n and len(tets) == T
    assert n + 2 * len(_edges(tets, n)) == nnzb
    vol = _signed_vol(rest, tets)
    assert (vol > 0).all()
    assert abs(vol.sum() - 1.0) < 1e-12


def test_kuhn_conforming():
    # every interior face is shared by exactly two tets, boundary faces by one
    rest, tets, _, _ = scenes.kuhn_cube(3)
    f = np.sort(np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]]), axis=1)
    _, cnt = np.unique(f, axis=0, return_counts=True)
    assert set(cnt.tolist()) <= {1, 2}
    assert (cnt == 1).sum() == 6 * 2 * 3 * 3  # 6 sides x 2 triangles x 3x3 quads


def test_gyroid_counts():
    s = scenes.gyroid_sphere()
    assert len(s["tets"]) == 219096 and len(s["rest"]) == 115533
    assert abs(s["rest"][:, 2].min() - 0.05) < 1e-12
    assert (_signed_vol(s["rest"], s["tets"]) > 0).all()


def test_inclusion_block_fields():
    s = scenes.inclusion_block(8, seed=3)
    assert set(np.unique(s["E"]).tolist()) <= {1e5, 1e10}
    t = s["dbc_targets"](5)
    top = s["rest"][s["dirichlet"], 2] > 0.5
    assert np.allclose(t[top, 2], 1.0 - 0.05)
    assert np.allclose(s["dbc_targets"](30)[top, 2], 0.9)


def test_batch_sizes():
    bs = scenes.batch_scenes(8, seed=1)
    assert len(bs) == 8
    for s in bs:
        assert (_signed_vol(s["rest"], s["tets"]) > 0).all()
        assert len(s["dirichlet"]) >= 3


@pytest.mark.parametrize("kind", ["random", "rcm"])
def test_vertex_renumbering_keeps_the_mesh(kind):
    s = scenes.inclusion_block(6, seed=2, steps=1)
    perm = scenes.vertex_order(s["rest"], s["tets"], kind, seed=1)
    assert sorted(perm.tolist()) == list(range(len(s["rest"])))
    t = scenes.permute_vertices(s, perm)
    assert np.array_equal(t["rest"][t["tets"]], s["rest"][s["tets"]])
    assert np.array_equal(t["rest"][t["dirichlet"]], s["rest"][s["dirichlet"]])
    assert np.array_equal(t["dbc_targets"](3), s["dbc_targets"](3))


def test_sliding_cube_starts_in_vertical_balance():
    s = scenes.sliding_cube(4)
    hs = s["halfspace"]
    z = s["rest"][:, 2]
    bottom = np.isclose(z, z.min())
    assert bottom.sum() == 25 and z.min() == pytest.approx(0.5 * hs["dhat"])
    from oracle import fem
    lam = hs["kappa"] * np.abs(fem.barrier_d1(z[bottom], hs["dhat"]))
    weight = 1000.0 * 0.2 ** 3 * 9.81
    assert lam.sum() == pytest.approx(weight, rel=1e-12)
