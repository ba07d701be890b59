"""Pins of the self-contact oracle (IPC point-triangle / edge-edge barriers
and time of impact)."""
import numpy as np
import pytest
import torch

import scenes
from oracle import selfcontact as sc

T = lambda a: torch.tensor(np.asarray(a, dtype=np.float64).ravel(), dtype=torch.float64)


def _rot(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return q * np.sign(np.linalg.det(q))


def test_surface_of_a_cube():
    rest, tets, _, _ = scenes.kuhn_cube(2)
    tris, edges, verts = sc.surface(tets)
    assert len(tris) == 12 * 2 * 2 and len(verts) == 26
    assert len(verts) - len(edges) + len(tris) == 2  # closed genus-0 surface
    # every surface edge borders exactly two surface triangles
    e = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [0, 2]]]), axis=1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    assert np.all(cnt == 2)


@pytest.mark.parametrize("p,d2", [((0.2, 0.2, 0.5), 0.25), ((0.5, -0.3, 0.4), 0.25), ((-0.3, -0.4, 0.0), 0.25),
                                  ((1.0, 1.0, 0.0), 0.5)])
def test_point_triangle_closed_forms(p, d2):
    tri = [(0, 0, 0), (1, 0, 0), (0, 1, 0)]
    assert float(sc.pt_dist2(T([p] + tri))) == pytest.approx(d2, rel=1e-14)


@pytest.mark.parametrize("seg,d2", [(((0, 0, 0), (1, 0, 0), (0.5, -1, 0.3), (0.5, 1, 0.3)), 0.09),
                                    (((0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0)), 1.0),
                                    (((0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)), 1.0),
                                    (((0, 0, 0), (1, 0, 0), (1.5, 1, 2), (3, 2, 2)), 0.25 + 1 + 4)])
def test_edge_edge_closed_forms(seg, d2):
    assert float(sc.ee_dist2(T(seg))) == pytest.approx(d2, rel=1e-14)


def test_distances_against_brute_force():
    rng = np.random.default_rng(0)
    uv = np.array([(u, v) for u in np.linspace(0, 1, 121) for v in np.linspace(0, 1, 121) if u + v <= 1])
    s = np.linspace(0, 1, 201)
    for _ in range(30):
        X = rng.standard_normal((4, 3))
        samples = X[1] + uv[:, :1] * (X[2] - X[1]) + uv[:, 1:] * (X[3] - X[1])
        brute = np.min(np.sum((samples - X[0]) ** 2, axis=1))
        d2 = float(sc.pt_dist2(T(X)))
        assert d2 <= brute + 1e-14 and brute - d2 <= 2e-3 * (1 + brute)
        A = X[0] + s[:, None] * (X[1] - X[0])
        B = X[2] + s[:, None] * (X[3] - X[2])
        brute = np.min(np.sum((A[:, None, :] - B[None, :, :]) ** 2, axis=2))
        d2 = float(sc.ee_dist2(T(X)))
        assert d2 <= brute + 1e-14 and brute - d2 <= 2e-3 * (1 + brute)


def _fd(kind, x12, dhat, eps, h=1e-7):
    f = lambda y: float(sc.pair_energy(kind, T(y), dhat, eps))
    g = np.zeros(12)
    for k in range(12):
        e = np.zeros(12)
        e[k] = h
        g[k] = (f(x12 + e) - f(x12 - e)) / (2 * h)
    return g


@pytest.mark.parametrize("kind", ["pt", "ee", "ee_parallel"])
def test_pair_derivatives_match_finite_differences_and_are_rigid_invariant(kind):
    rng = np.random.default_rng({"pt": 1, "ee": 2, "ee_parallel": 3}[kind])
    dhat = 0.1
    if kind == "pt":
        X = np.array([(0.2, 0.3, 0.04), (0, 0, 0), (1, 0, 0), (0, 1, 0)]) + 1e-3 * rng.standard_normal((4, 3))
        eps = None
        k = "pt"
    else:
        k = "ee"
        X = np.array([(0, 0, 0), (1, 0, 0), (0.5, -0.5, 0.05), (0.5, 0.5, 0.05)])
        if kind == "ee_parallel":  # nearly parallel: the mollifier is active
            X = np.array([(0, 0, 0), (1, 0, 0), (0.1, 0.02, 0.05), (1.1, 0.0, 0.05)])
        X = X + 1e-4 * rng.standard_normal((4, 3))
        R = X.copy()
        eps = 1e-3 * np.sum((R[1] - R[0]) ** 2) * np.sum((R[3] - R[2]) ** 2)
    x12 = X.ravel()
    e, g, H = sc.pair_derivatives(k, x12, dhat, eps, project=False)
    assert e > 0
    gfd = _fd(k, x12, dhat, eps)
    assert np.abs(g - gfd).max() <= 1e-6 * np.abs(g).max()
    # Hessian against differences of the gradient
    h = 1e-6
    Hfd = np.zeros((12, 12))
    for j in range(12):
        d = np.zeros(12)
        d[j] = h
        Hfd[:, j] = (sc.pair_derivatives(k, x12 + d, dhat, eps, project=False)[1] -
                     sc.pair_derivatives(k, x12 - d, dhat, eps, project=False)[1]) / (2 * h)
    assert np.abs(H - Hfd).max() <= 1e-5 * np.abs(H).max()
    # rigid motions leave the energy unchanged; gradients sum to zero
    Q = _rot(7)
    Y = X @ Q.T + np.array([0.3, -2.0, 1.1])
    assert float(sc.pair_energy(k, T(Y), dhat, eps)) == pytest.approx(e, rel=1e-10)
    assert np.abs(g.reshape(4, 3).sum(axis=0)).max() <= 1e-9 * np.abs(g).max()
    # the projected Hessian is PSD
    Hp = sc.pair_derivatives(k, x12, dhat, eps, project=True)[2]
    assert np.linalg.eigvalsh(Hp).min() >= -1e-10 * np.abs(Hp).max()
    if kind == "ee_parallel":
        c = np.sum(np.cross(X[1] - X[0], X[3] - X[2]) ** 2)
        assert c < eps


def test_mollifier_closed_form_and_smoothness():
    eps = 0.3
    m = lambda c: float(sc.mollifier(torch.tensor(c, dtype=torch.float64), eps))
    assert m(0.0) == 0.0 and m(eps) == pytest.approx(1.0) and m(2 * eps) == 1.0
    assert m(0.15) == pytest.approx((2 - 0.5) * 0.5)
    # C1 at eps_x: the one-sided slope from below vanishes like h / eps^2
    for h in (1e-4, 1e-6):
        assert abs((m(eps) - m(eps - h)) / h) <= 2.0 * h / eps ** 2


def test_energy_vanishes_beyond_dhat():
    X = np.array([(0.2, 0.3, 0.2), (0, 0, 0), (1, 0, 0), (0, 1, 0)])
    assert float(sc.pair_energy("pt", T(X), 0.1)) == 0.0
    assert float(sc.pair_energy("pt", T(X), 0.25)) > 0.0


def _two_cubes(gap):
    rest, tets, _, _ = scenes.kuhn_cube(1)
    top = rest + np.array([0.15, 0.1, 1.0 + gap])
    return np.concatenate([rest, top]), np.concatenate([tets, tets + len(rest)])


def test_assembled_terms_on_two_cubes():
    rest, tets = _two_cubes(0.02)
    x = rest + 1e-3 * np.random.default_rng(4).standard_normal(rest.shape)
    surf = sc.surface(tets)
    pairs = sc.active_pairs(x, surf, 0.05)
    assert len(pairs[0]) > 0 and len(pairs[1]) > 0
    # only pairs between the two bodies are this close
    assert all((q[0] < 8) != (q[1] < 8) for q in pairs[0])
    E, g, H = sc.contact_terms(x, rest, pairs, 0.05, 10.0)
    assert E > 0
    assert np.abs(g.sum(axis=0)).max() <= 1e-9 * np.abs(g).max()  # no net force
    assert np.abs(H - H.T).max() == 0.0
    assert np.linalg.eigvalsh(H).min() >= -1e-9 * np.abs(H).max()
    # gradient against central differences of the total (same pair set)
    k, h = 11, 1e-7
    for comp in range(3):
        xp, xm = x.copy(), x.copy()
        xp[k, comp] += h
        xm[k, comp] -= h
        fd = (sc.contact_terms(xp, rest, pairs, 0.05, 10.0, project=False)[0] -
              sc.contact_terms(xm, rest, pairs, 0.05, 10.0, project=False)[0]) / (2 * h)
        assert fd == pytest.approx(g[k, comp], rel=1e-6, abs=1e-9 * np.abs(g).max())


def test_time_of_impact_analytic_cases():
    tri = np.array([(0, 0, 0), (1, 0, 0), (0, 1, 0)], dtype=float)
    # a point falling onto the triangle: contact half way
    x = np.concatenate([[0.2, 0.2, 1.0], tri.ravel()])
    p = np.concatenate([[0.0, 0.0, -2.0], np.zeros(9)])
    assert sc.toi("pt", x, p) == pytest.approx(0.5, abs=1e-12)
    # the triangle rising to meet it: contact at 1/4
    p2 = np.concatenate([[0.0, 0.0, -2.0], np.tile([0.0, 0.0, 2.0], 3)])
    assert sc.toi("pt", x, p2) == pytest.approx(0.25, abs=1e-12)
    # falling beside the triangle: no contact
    x3 = np.concatenate([[0.8, 0.8, 1.0], tri.ravel()])
    assert sc.toi("pt", x3, p) is None
    # an edge falling onto a crossing edge
    e = np.array([(0, 0, 1.0), (1, 0, 1.0), (0.5, -1, 0), (0.5, 1, 0)]).ravel()
    pe = np.array([(0, 0, -4.0), (0, 0, -4.0), (0, 0, 0), (0, 0, 0)]).ravel()
    assert sc.toi("ee", e, pe) == pytest.approx(0.25, abs=1e-12)
    # passing beyond the end of the other edge: no contact
    e2 = np.array([(0, 2.0, 1.0), (1, 2.0, 1.0), (0.5, -1, 0), (0.5, 1, 0)]).ravel()
    assert sc.toi("ee", e2, pe) is None


def test_time_of_impact_against_sampled_distance():
    rng = np.random.default_rng(5)
    found = 0
    for _ in range(40):
        X = rng.uniform(-1, 1, (4, 3))
        P = rng.uniform(-2, 2, (4, 3))
        for kind, dist in (("pt", sc.pt_dist2), ("ee", sc.ee_dist2)):
            t = sc.toi(kind, X.ravel(), P.ravel())
            ts = np.linspace(0, 1, 2001)
            d = np.array([float(dist(T(X + s * P))) for s in ts])
            if t is None:
                assert d.min() > 0.0
                continue
            found += 1
            assert float(dist(T(X + t * P))) <= 1e-16
            before = ts < t - 1e-3
            assert np.all(d[before] > 0.0)
    assert found > 5


def test_additive_ccd_is_conservative():
    rng = np.random.default_rng(6)
    hits = 0
    for _ in range(60):
        X = rng.uniform(-1, 1, (4, 3))
        P = rng.uniform(-2, 2, (4, 3))
        for kind, dist in (("pt", sc.pt_dist2), ("ee", sc.ee_dist2)):
            t_exact = sc.toi(kind, X.ravel(), P.ravel())
            hit, t = sc.accd(kind, X.ravel(), P.ravel(), s=0.1)
            if t_exact is not None:
                assert hit and t <= t_exact
                hits += 1
            if hit:
                d0 = np.sqrt(float(dist(T(X))))
                dt = np.sqrt(float(dist(T(X + t * P))))
                assert dt >= 0.1 * d0 * (1 - 1e-12)  # separated by at least s times the start gap
    assert hits > 5
    # the falling point: hit before t = 0.5, within the last step's margin
    tri = np.array([(0, 0, 0), (1, 0, 0), (0, 1, 0)], dtype=float)
    x = np.concatenate([[0.2, 0.2, 1.0], tri.ravel()])
    p = np.concatenate([[0.0, 0.0, -2.0], np.zeros(9)])
    hit, t = sc.accd("pt", x, p, s=0.1)
    assert hit and 0.45 <= t < 0.5
    # a common translation is no relative motion
    hit, t = sc.accd("pt", x, np.tile([0.0, 0.0, -2.0], 4))
    assert not hit and t == 1.0
