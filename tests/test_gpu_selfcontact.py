"""GPU additive CCD of self-contact primitive pairs against the oracle: the
same algorithm step for step (times within round-off, same hit flags), and
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
    assert same >= 0.98 * len(kind)
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
