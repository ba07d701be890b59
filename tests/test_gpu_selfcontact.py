"""GPU additive CCD of self-contact primitive pairs against the oracle: the
same algorithm step for step (times within round-off, same hit flags;
where the two end differently the oracle's run passes one of its decision
thresholds within a round-off margin), and
the properties that make it a filter: never later than the exact time of
impact, the pair still separated at the returned time."""
import numpy as np
import pytest
import torch

from oracle import selfcontact as sc
from tests.gpu_util import device, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def _cases(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (n, 4, 3))
    P = rng.uniform(-2, 2, (n, 4, 3))
    kind = rng.integers(0, 2, n).astype(np.int32)
    return kind, X, P


def test_accd_matches_oracle_and_is_conservative(dev):
    from paper_2508_13386_amd import ms
    kind, X, P = _cases(400, 11)
    # a few exact impacts and pure translations among them
    tri = np.array([(0, 0, 0), (1, 0, 0), (0, 1, 0)], dtype=float)
    X[0] = np.concatenate([[[0.2, 0.2, 1.0]], tri])
    P[0] = np.array([(0, 0, -2.0), (0, 0, 0), (0, 0, 0), (0, 0, 0)])
    kind[0] = 0
    P[1] = np.tile([0.3, -0.2, 0.5], (4, 1))
    say("accd pairs", len(kind))
    hit, t = ms.ms_contact_toi(dev, kind, X.reshape(-1, 12), P.reshape(-1, 12), s=0.1, t_max=1.0)
    same = 0
    for q in range(len(kind)):
        k = "pt" if kind[q] == 0 else "ee"
        oh, ot = sc.accd(k, X[q].ravel(), P[q].ravel(), s=0.1, t_max=1.0)
        if bool(hit[q]) == oh and abs(t[q] - ot) <= 1e-9 * max(ot, 1e-300):
            same += 1
        else:
            # a different end is allowed only where the oracle's own run
            # clears one of its decisions by a round-off margin
            margin = sc.accd_margin(k, X[q].ravel(), P[q].ravel(), s=0.1, t_max=1.0)
            say("  pair", q, k, "GPU", bool(hit[q]), t[q], "oracle", oh, ot, "decision margin", margin)
            assert margin <= 1e-9, q
        # the filter's guarantees hold for every pair
        exact = sc.toi(k, X[q].ravel(), P[q].ravel())
        if exact is not None:
            assert hit[q] and t[q] <= exact
        if hit[q]:
            dist = sc.pt_dist2 if k == "pt" else sc.ee_dist2
            d0 = np.sqrt(float(dist(torch.tensor(X[q].ravel()))))
            dt = np.sqrt(float(dist(torch.tensor((X[q] + t[q] * P[q]).ravel()))))
            assert dt >= 0.1 * d0 * (1 - 1e-9)
    say("  same as the oracle step for step:", same, "of", len(kind), "| hits", int(hit.sum()))
    assert hit[0] and 0.45 <= t[0] < 0.5
    assert not hit[1] and t[1] == 1.0


def test_accd_rejects_bad_arguments(dev):
    from paper_2508_13386_amd import ms
    kind, X, P = _cases(4, 1)
    with pytest.raises(ms.MSError):
        ms.ms_contact_toi(dev, np.array([0, 2, 0, 1], np.int32), X.reshape(-1, 12), P.reshape(-1, 12))
    with pytest.raises(ms.MSError):
        ms.ms_contact_toi(dev, kind, X.reshape(-1, 12), P.reshape(-1, 12), s=1.5)
    Xn = X.copy()
    Xn[0, 0, 0] = np.nan
    with pytest.raises(ms.MSError):
        ms.ms_contact_toi(dev, kind, Xn.reshape(-1, 12), P.reshape(-1, 12))


def _two_cubes(N, gap, seed):
    import scenes
    rest, tets, _, _ = scenes.kuhn_cube(N)
    top = rest + np.array([0.15, 0.1, 1.0 + gap])
    rest2 = np.concatenate([rest, top])
    tets2 = np.concatenate([tets, tets + len(rest)])
    x = rest2 + 1e-3 * np.random.default_rng(seed).standard_normal(rest2.shape)
    return x, tets2


@pytest.mark.parametrize("N,gap,cell", [(2, 0.02, 0.0), (2, 0.02, 0.07), (3, 0.01, 0.0), (2, 0.5, 0.0)])
def test_contact_pairs_match_brute_force(dev, N, gap, cell):
    from paper_2508_13386_amd import ms
    x, tets = _two_cubes(N, gap, N)
    tris, edges, verts = sc.surface(tets)
    dhat = 0.05
    say("pairs: surface", len(verts), "verts", len(tris), "tris", len(edges), "edges; cell", cell)
    pt, ee = ms.ms_contact_pairs(dev, x, verts, tris, edges, dhat, cell)
    opt, oee = sc.active_pairs(x, (tris, edges, verts), dhat)
    got_pt = {(int(v), *map(int, tris[t])) for v, t in pt}
    got_ee = {(*map(int, edges[i]), *map(int, edges[j])) for i, j in ee}
    say("  gpu", len(got_pt), "PT", len(got_ee), "EE | oracle", len(opt), "PT", len(oee), "EE")
    assert len(got_pt) == len(pt) and len(got_ee) == len(ee)  # no duplicates
    assert np.all(np.diff(pt[:, 0].astype(np.int64) * 2**32 + pt[:, 1]) > 0) if len(pt) > 1 else True
    assert all(i < j for i, j in ee)

    def borderline(kind, q):
        d2 = float((sc.pt_dist2 if kind == "pt" else sc.ee_dist2)(torch.tensor(x[list(q)].ravel())))
        return abs(d2 - dhat * dhat) <= 1e-12 * dhat * dhat

    assert {q for q in got_pt ^ set(opt) if not borderline("pt", q)} == set()
    assert {q for q in got_ee ^ set(oee) if not borderline("ee", q)} == set()
    if gap < 0.1:
        assert len(opt) > 0 and len(oee) > 0
