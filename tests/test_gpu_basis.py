"""The basis build's local biharmonic solves as dense Cholesky on the GPU
(ms_build_basis with gpu_min_unknowns): the weights equal the host build's
(same partitioning, envelope Cholesky) and the oracle's (basis_weights given
the library's partitioning) within the tolerance the local operator's
conditioning allows (as in tests/test_oracle_basis.py)."""
import numpy as np
import pytest

import scenes
from oracle import basis
from tests.gpu_util import device, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scene,m,dbc,rtol,atol", [("plain_cube", 8, False, 1e-9, 1e-12),
                                                   ("inclusion_block", 10, True, 0.0, 2e-5)])
def test_gpu_local_solves_match_host_and_oracle(scene, m, dbc, rtol, atol):
    from paper_2508_13386_amd import ms
    dev = device()
    s = scenes.plain_cube(6, seed=1) if scene == "plain_cube" else scenes.inclusion_block(8, seed=2, steps=1)
    d = s["dirichlet"] if dbc else np.zeros(0, np.int32)
    c = ms.Context(dev)
    c.ms_upload_mesh(s["rest"], s["tets"])
    c.ms_upload_material(s["E"], s["nu"], s["rho"])
    if len(d):
        c.ms_set_dirichlet(d, s["rest"][d])
    c.ms_set_state(s["x0"], s["v0"])
    c.ms_build_basis(n_handles=m, seed=5, n_threads=2, gpu_min_unknowns=32)
    gsolves, secs = c.ms_get_basis_stats()
    b = c.ms_get_basis()
    c.close()
    host = ms.ms_basis_compute(s["rest"], s["tets"], s["E"], d, n_handles=m, seed=5, n_threads=2)
    say(scene, "local solves on the GPU", gsolves, "of", b["m"] + (1 if len(d) else 0), "build", round(secs, 3), "s")
    assert gsolves >= b["m"]
    assert np.array_equal(b["part"], host["part"])
    assert np.array_equal(b["vptr"], host["vptr"]) and np.array_equal(b["vhandle"], host["vhandle"])
    assert np.allclose(b["vphi"], host["vphi"], rtol=rtol, atol=atol)
    out = basis.basis_weights(s["rest"], s["tets"], s["E"], d, b["part"])
    assert np.abs(b["origins"] - out["origins"]).max() <= 1e-12
    for v in range(len(s["rest"])):
        row = [(int(b["vhandle"][k]), float(b["vphi"][k])) for k in range(b["vptr"][v], b["vptr"][v + 1])]
        orc = out["rows"][v]
        assert [i for i, _ in row] == [i for i, _ in orc], v
        assert np.allclose([p for _, p in row], [p for _, p in orc], rtol=rtol, atol=atol), v


def test_gpu_basis_of_the_bench_block_matches_host():
    """The 32^3 heterogeneous block with its Dirichlet faces, 192 handles: the
    large Dirichlet subdomain (about 27.5 K unknowns) is factored on the GPU
    by default; the weights agree with the all-host build."""
    from paper_2508_13386_amd import ms
    dev = device()
    s = scenes.inclusion_block(32, seed=0, steps=3)
    c = ms.context_from_scene(dev, s)
    c.ms_build_basis(n_handles=192, oversample=1.0)
    g, t_gpu = c.ms_get_basis_stats()
    b = c.ms_get_basis()
    c.ms_build_basis(n_handles=192, oversample=1.0, gpu_min_unknowns=0)
    g0, t_host = c.ms_get_basis_stats()
    h = c.ms_get_basis()
    c.close()
    say("bench block basis: GPU solves", g, "build", round(t_gpu, 2), "s | host only", round(t_host, 2), "s")
    assert g >= 1 and g0 == 0
    assert np.array_equal(b["part"], h["part"])  # device and host nearest-seed searches agree
    assert np.array_equal(b["vptr"], h["vptr"]) and np.array_equal(b["vhandle"], h["vhandle"])
    err = np.abs(b["vphi"] - h["vphi"]).max()
    say("max weight difference", err)
    assert err <= 2e-5


@pytest.mark.parametrize("kw", [dict(n_handles=40, seed=1, oversample=1.5), dict(n_handles=27, lattice_seeding=1)])
def test_device_voronoi_partitioning_equals_host(kw):
    """kmeans++ seeding with oversampling and pruning, and lattice seeding:
    with the nearest-seed searches on the GPU (every local solve kept on the
    host) the basis equals the host-only build exactly."""
    from paper_2508_13386_amd import ms
    dev = device()
    s = scenes.inclusion_block(12, seed=3, steps=3)
    c = ms.context_from_scene(dev, s)
    c.ms_build_basis(gpu_min_unknowns=10 ** 9, n_threads=2, **kw)
    g, secs = c.ms_get_basis_stats()
    b = c.ms_get_basis()
    c.close()
    h = ms.ms_basis_compute(s["rest"], s["tets"], s["E"], s["dirichlet"], n_threads=2, **kw)
    say(kw, "partitions", b["m"], "GPU solves", g, "build", round(secs, 3), "s")
    assert g == 0
    assert np.array_equal(b["part"], h["part"])
    for k in ("vptr", "vhandle", "vphi", "origins"):
        assert np.array_equal(b[k], h[k]), k
