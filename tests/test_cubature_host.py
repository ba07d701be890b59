"""The library's host cubature fit (Alg. 3, no device involved) checked by
the oracle's moment conditions (CPU only)."""
import numpy as np
import pytest

import scenes
from oracle import cubature as cub
from tests.test_oracle_cubature import _basis, _partition


@pytest.mark.parametrize("N,k,seed", [(4, 2, 0), (6, 3, 1)])
def test_host_fit_meets_the_moment_conditions(N, k, seed):
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(N, seed=seed)
    part = _partition(s["rest"], s["tets"], k)
    B = _basis(s, part)
    t, w, res = ms.ms_cubature_compute(s["rest"], s["tets"], part, B, tol=1e-9, n_init=8, n_add=8, seed=seed,
                                       n_threads=2)
    assert np.all(np.diff(t) > 0) and np.all(w > 0.0)
    assert len(t) < len(s["tets"])
    r = cub.moment_residuals(s["rest"], s["tets"], part, B, t, w)
    assert max(r.values()) <= 1e-9
    assert res == pytest.approx(max(r.values()), rel=1e-3, abs=1e-15)
    Ue = cub.element_values(s["tets"], B["vptr"], B["vhandle"], B["vphi"], B["m"])
    for p in np.unique(part):
        ids = np.nonzero(part == p)[0]
        A, _, _ = cub.moment_system(Ue[ids], np.ones(len(ids)))
        assert np.count_nonzero(part[t] == p) <= np.linalg.matrix_rank(A)
    # same seed, same result (thread count does not matter)
    t2, w2, _ = ms.ms_cubature_compute(s["rest"], s["tets"], part, B, tol=1e-9, n_init=8, n_add=8, seed=seed,
                                       n_threads=1)
    assert np.array_equal(t, t2) and np.array_equal(w, w2)


def test_host_fit_single_constant_function():
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(3, seed=0)
    n = len(s["rest"])
    part = _partition(s["rest"], s["tets"])
    B = dict(m=1, vptr=np.arange(n + 1), vhandle=np.zeros(n, np.int32), vphi=np.ones(n))
    vol = cub.tet_volumes(s["rest"], s["tets"])
    t, w, _ = ms.ms_cubature_compute(s["rest"], s["tets"], part, B, n_init=4, n_add=4, seed=2)
    for p in np.unique(part):
        sel = part[t] == p
        assert sel.sum() == 1
        assert w[sel][0] == pytest.approx(vol[part == p].sum(), rel=1e-12)


def test_host_fit_rejects_bad_arguments():
    from paper_2508_13386_amd import ms
    s = scenes.plain_cube(3, seed=0)
    part = _partition(s["rest"], s["tets"])
    B = _basis(s, part)
    bad = part.copy()
    bad[0] = -1
    with pytest.raises(ms.MSError):
        ms.ms_cubature_compute(s["rest"], s["tets"], bad, B)
    with pytest.raises(ms.MSError):
        ms.ms_cubature_compute(s["rest"], s["tets"], part, B, n_add=0)
    with pytest.raises(ms.MSError):
        ms.ms_cubature_compute(s["rest"], s["tets"], part, dict(B, m=1))
