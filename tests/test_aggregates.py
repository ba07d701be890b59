"""Host logic of the aggregate smoother's vertex aggregation
(ms_aggregates_compute, no device): on a regular grid the aggregates are
the 2 x 2 x 2 vertex blocks (ragged at an odd side), every vertex belongs to
exactly one aggregate, crowded bins split into groups of at most eight, and
malformed input is rejected."""
import numpy as np
import pytest

import scenes
from paper_2508_13386_amd import ms


def _graph(n, tets):
    """Vertex graph (CSR, self entries included) of a tet mesh."""
    pairs = set()
    for t in tets:
        for a in t:
            for b in t:
                pairs.add((int(a), int(b)))
    for v in range(n):
        pairs.add((v, v))
    p = np.array(sorted(pairs), dtype=np.int64)
    row_ptr = np.searchsorted(p[:, 0], np.arange(n + 1)).astype(np.int32)
    return row_ptr, p[:, 1].astype(np.int32)


def _check_partition(agg, n):
    members = agg[agg >= 0]
    assert np.array_equal(np.sort(members), np.arange(n))  # every vertex exactly once
    assert ((agg >= 0).sum(axis=1) >= 1).all()
    # padding only at the end of a group
    for row in agg:
        k = (row >= 0).sum()
        assert (row[:k] >= 0).all() and (row[k:] == -1).all()


@pytest.mark.parametrize("N", [1, 4, 7])
def test_regular_grid_gives_2x2x2_blocks(N):
    rest, tets, _, _ = scenes.kuhn_cube(N)
    n = len(rest)
    row_ptr, col = _graph(n, tets)
    agg = ms.ms_aggregates_compute(rest, row_ptr, col)
    _check_partition(agg, n)
    ijk = np.rint(rest * N).astype(int)
    blocks = {tuple(sorted(r[r >= 0].tolist())) for r in agg}
    expect = {}
    for v in range(n):
        expect.setdefault(tuple(ijk[v] // 2), []).append(v)
    assert blocks == {tuple(sorted(vs)) for vs in expect.values()}
    nb = (N + 2) // 2  # blocks per axis for N + 1 vertices
    assert len(agg) == nb ** 3
    sizes = np.sort((agg >= 0).sum(axis=1))
    if N % 2 == 1:
        assert (sizes == 8).all()  # an even vertex count per axis: full blocks only
    else:
        assert sizes.max() == 8 and sizes.min() == 1  # the odd side leaves ragged blocks


def test_crowded_bins_split_in_vertex_order():
    """A unit edge sets the bin width (2); twenty vertices inside a 0.5-cube
    far away, joined to the mesh only by long edges, share one bin and form
    groups of 8, 8 and 4 in vertex order."""
    rng = np.random.default_rng(0)
    rest = np.vstack([[[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]], 10.0 + 0.5 * rng.random((20, 3))])
    n = len(rest)
    rows = [list(range(n)), [0, 1]] + [[0, v] for v in range(2, n)]
    row_ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    col = np.concatenate([np.array(r) for r in rows]).astype(np.int32)
    agg = ms.ms_aggregates_compute(rest, row_ptr, col)
    _check_partition(agg, n)
    groups = [r[r >= 0].tolist() for r in agg]
    assert groups == [[0, 1], list(range(2, 10)), list(range(10, 18)), list(range(18, 22))]


def test_rejects_malformed_input():
    rest, tets, _, _ = scenes.kuhn_cube(2)
    n = len(rest)
    row_ptr, col = _graph(n, tets)
    bad = rest.copy()
    bad[3, 1] = np.nan
    with pytest.raises(ms.MSError) as e:
        ms.ms_aggregates_compute(bad, row_ptr, col)
    assert e.value.code == ms.MS_E_NONFINITE
    c2 = col.copy()
    c2[5] = n
    with pytest.raises(ms.MSError) as e:
        ms.ms_aggregates_compute(rest, row_ptr, c2)
    assert e.value.code == ms.MS_E_MESH
    r2 = row_ptr.copy()
    r2[0] = 1
    with pytest.raises(ms.MSError) as e:
        ms.ms_aggregates_compute(rest, r2, col)
    assert e.value.code == ms.MS_E_MESH
    with pytest.raises(ms.MSError) as e:
        ms.ms_aggregates_compute(np.zeros((0, 3)), np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert e.value.code == ms.MS_E_ARG
