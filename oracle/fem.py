"""Incremental potential of the implicit Euler timestep (FP64, CPU oracle).

Test infrastructure only.  Follows Sec. 3.1 of the paper:
  E(x) = K(x) + alpha h^2 (Psi(x) + B(x) + D(x)),  K = 1/2 ||x - x~||_M^2,
  implicit Euler: x~ = x^t + h v^t, alpha = 1, v^{t+1} = (x^{t+1} - x^t)/h;
  BDF2: x~ = 4/3 x^t - 1/3 x^{t-1} + h (8 v^t - 2 v^{t-1}) / 9, alpha = 4/9,
        v^{t+1} = (3 x^{t+1} - 4 x^t + x^{t-1}) / (2h).

Readings where the paper is silent (each also listed in the design notes):
  * Psi is the stable Neo-Hookean energy
        Psi(F) = mu/2 (tr F^T F - 3) - mu (J - 1) + lam'/2 (J - 1)^2,
    mu = E / (2(1+nu)), lam' = E nu / ((1+nu)(1-2nu)) + mu, chosen so the
    small-strain limit is linear elasticity with (E, nu).  The paper names a
    "non-inverting Neo-Hookean" model (Sec. 4) without a formula.
  * M is the lumped mass m_v = sum_{e ni v} rho_e V_e / 4.
  * Gravity enters as the potential -sum_v m_v g . x_v inside the h^2 term.
  * B is the IPC log barrier b(d) = -(d - dhat)^2 ln(d / dhat) for 0 < d < dhat
    (Li et al. 2020) on the signed distance d_v = n . x_v - c of every vertex
    to a rigid half-space, scaled by a stiffness kappa.
  * D is lagged Coulomb friction against the half-space in the IPC form (the
    paper's D(x) term; off unless the half-space has mu > 0):
        D(x) = sum_v mu lambda_v f0(|u_v|),  u_v = P (x_v - x_v^t),  P = I - n n^T,
    with the normal force lambda_v = kappa |b'(d_v(x^t))| frozen at the start
    of the step and the smoothed magnitude f0(y) = y for y >= eps_v h, else
    -y^3 / (3 (eps_v h)^2) + y^2 / (eps_v h) + eps_v h / 3 (C1 at eps_v h).
  * The element Hessian is made PSD by clamping the negative eigenvalues of
    the 9x9 deformation-gradient Hessian (the usual IPC practice); this
    changes Newton iterates only, not the minimiser.

Pinned by tests/test_oracle_fem.py: central finite differences of every term,
the rest state, rigid-motion invariance, closed forms of the barrier.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class MeshError(ValueError):
    """A rest tetrahedron has non-positive volume."""


# Levi-Civita symbol: det F = eps_ijk F_i0 F_j1 F_k2.
EPS = np.zeros((3, 3, 3))
for _i, _j, _k in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    EPS[_i, _j, _k] = 1.0
    EPS[_i, _k, _j] = -1.0


def lame(E, nu):
    """(mu, lam') of the stable Neo-Hookean parametrisation."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam + mu


class Body:
    """Rest-state quantities of a tet mesh: volumes, shape-function gradients,
    lumped masses, material."""

    def __init__(self, rest, tets, E, nu, rho):
        self.rest = np.asarray(rest, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        X = self.rest[self.tets]  # [T,4,3]
        Dm = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))  # columns = edges
        vol = np.linalg.det(Dm) / 6.0
        if self.tets.size and not (vol > 0).all():
            raise MeshError("non-positive rest volume at tet %d" % int(np.argmin(vol)))
        Dminv = np.linalg.inv(Dm)
        beta = np.empty((len(self.tets), 4, 3))
        beta[:, 1:, :] = Dminv  # grad of barycentric coordinate a (row a-1 of Dm^-1)
        beta[:, 0, :] = -Dminv.sum(axis=1)
        self.vol = vol
        self.beta = beta  # F = sum_a x_a (x) beta_a
        self.mu, self.lam = lame(E, nu)
        rho = np.asarray(rho, dtype=np.float64)
        n = len(self.rest)
        self.n = n
        self.mass = np.zeros(n)
        np.add.at(self.mass, self.tets.ravel(), np.repeat(rho * vol / 4.0, 4))

    def deformation_gradient(self, x):
        return np.einsum("tai,taj->tij", x[self.tets], self.beta)


# ----------------------------------------------------------------------------
# Stable Neo-Hookean density and its derivatives w.r.t. F (batched over tets).
# ----------------------------------------------------------------------------
def snh_psi(F, mu, lam):
    J = np.linalg.det(F)
    Ic = np.einsum("tij,tij->t", F, F)
    return 0.5 * mu * (Ic - 3.0) - mu * (J - 1.0) + 0.5 * lam * (J - 1.0) ** 2


def cofactor(F):
    """dJ/dF: cof_ip = 1/2 eps_ijk eps_pqr F_jq F_kr."""
    return 0.5 * np.einsum("ijk,pqr,tjq,tkr->tip", EPS, EPS, F, F, optimize=True)


def snh_P(F, mu, lam):
    J = np.linalg.det(F)
    s = lam * (J - 1.0) - mu
    return mu[:, None, None] * F + s[:, None, None] * cofactor(F)


def snh_dPdF(F, mu, lam):
    """9x9 Hessian d^2 Psi / dF_ip dF_jq, flattened with row index 3 i + p."""
    T = len(F)
    J = np.linalg.det(F)
    s = lam * (J - 1.0) - mu
    G = cofactor(F).reshape(T, 9)
    HJ = np.einsum("ijk,pqr,tkr->tipjq", EPS, EPS, F, optimize=True).reshape(T, 9, 9)
    return (mu[:, None, None] * np.eye(9)[None] + lam[:, None, None] * G[:, :, None] * G[:, None, :]
            + s[:, None, None] * HJ)


def project_psd(A):
    """Clamp negative eigenvalues of a batch of symmetric matrices to zero."""
    w, V = np.linalg.eigh(A)
    return np.einsum("tik,tk,tjk->tij", V, np.maximum(w, 0.0), V)


# ----------------------------------------------------------------------------
# IPC log barrier and its derivatives in the distance d.
# ----------------------------------------------------------------------------
def barrier(d, dhat):
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -((dm - dhat) ** 2) * np.log(dm / dhat)
    out[d <= 0] = np.inf
    return out


def barrier_d1(d, dhat):
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -2.0 * (dm - dhat) * np.log(dm / dhat) - (dm - dhat) ** 2 / dm
    return out


def barrier_d2(d, dhat):
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -2.0 * np.log(dm / dhat) - 4.0 * (dm - dhat) / dm + (dm - dhat) ** 2 / dm ** 2
    return out


# ----------------------------------------------------------------------------
# Smoothed friction magnitude f0 and its derivatives in y = |u| (eh = eps_v h).
# ----------------------------------------------------------------------------
def friction_f0(y, eh):
    y = np.asarray(y, dtype=np.float64)
    out = y.copy()
    m = y < eh
    ym = y[m]
    out[m] = -ym ** 3 / (3.0 * eh * eh) + ym * ym / eh + eh / 3.0
    return out


def friction_f1(y, eh):
    """f0'(y): 1 beyond eh, -y^2/eh^2 + 2y/eh below (0 at rest)."""
    y = np.asarray(y, dtype=np.float64)
    out = np.ones_like(y)
    m = y < eh
    ym = y[m]
    out[m] = -ym * ym / (eh * eh) + 2.0 * ym / eh
    return out


def friction_f2(y, eh):
    """f0''(y)."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(y)
    m = y < eh
    out[m] = -2.0 * y[m] / (eh * eh) + 2.0 / eh
    return out


# ----------------------------------------------------------------------------
# The incremental potential of one implicit Euler step.
# ----------------------------------------------------------------------------
class StepProblem:
    """E(x) of one implicit Euler step (Eq. IP with alpha = 1)."""

    def __init__(self, body: Body, x_t, v_t, h, gravity, halfspace=None, prev=None, selfcontact=None):
        """prev = (x^{t-1}, v^{t-1}) selects BDF2: x~ = 4/3 x^t - 1/3 x^{t-1} +
        8/9 h v^t - 2/9 h v^{t-1} and the weight alpha = 4/9 on the h^2 terms
        (Sec. 3.1 names BDF2 beside implicit Euler; the scheme is the standard
        second-order backward difference in x and v).  None: implicit Euler.
        selfcontact = dict(dhat, kappa) adds IPC self-contact between the
        body's surface primitives (term C: h^2 kappa times the pair barriers
        of oracle.selfcontact over the pairs closer than dhat at x)."""
        self.b = body
        self.sc = None
        if selfcontact is not None:
            from . import selfcontact as scm
            self.sc = dict(dhat=float(selfcontact["dhat"]), kappa=float(selfcontact["kappa"]),
                           surf=scm.surface(body.tets))
        self.h = float(h)
        self.x_t = np.asarray(x_t, dtype=np.float64)
        v_t = np.asarray(v_t, dtype=np.float64)
        if prev is None:
            self.alpha = 1.0
            self.xtilde = self.x_t + self.h * v_t
        else:
            xp, vp = (np.asarray(a, dtype=np.float64) for a in prev)
            self.alpha = 4.0 / 9.0
            self.xtilde = (4.0 * self.x_t - xp) / 3.0 + self.h * (8.0 * v_t - 2.0 * vp) / 9.0
        self.gravity = np.asarray(gravity, dtype=np.float64)
        self.hs = halfspace
        # lagged friction: mu lambda_v from the contact forces at x^t
        self.fric = None
        if halfspace is not None and float(halfspace.get("mu", 0.0)) > 0.0:
            lam = float(halfspace["kappa"]) * np.abs(barrier_d1(self._dist(self.x_t), float(halfspace["dhat"])))
            nrm = np.asarray(halfspace["normal"], dtype=np.float64)
            self.fric = dict(mulam=float(halfspace["mu"]) * lam, eh=float(halfspace["eps_v"]) * self.h,
                             P=np.eye(3) - np.outer(nrm, nrm))

    # -- parts ---------------------------------------------------------------
    def _dist(self, x):
        n = np.asarray(self.hs["normal"], dtype=np.float64)
        return x @ n - float(self.hs["offset"])

    def energy_parts(self, x):
        b, h2 = self.b, self.alpha * self.h * self.h
        dx = x - self.xtilde
        K = 0.5 * float((b.mass[:, None] * dx * dx).sum())
        F = b.deformation_gradient(x)
        Psi = float((b.vol * snh_psi(F, b.mu, b.lam)).sum())
        G = -float((b.mass[:, None] * self.gravity[None, :] * x).sum())
        Bv = 0.0
        if self.hs is not None:
            Bv = float(self.hs["kappa"]) * float(barrier(self._dist(x), float(self.hs["dhat"])).sum())
        Dv = 0.0
        if self.fric is not None:
            y = np.linalg.norm((x - self.x_t) @ self.fric["P"], axis=1)
            Dv = float((self.fric["mulam"] * friction_f0(y, self.fric["eh"])).sum())
        Cv = 0.0
        if self.sc is not None:
            Cv = self._contact(x, project=True)[0]
        return dict(K=K, Psi=h2 * Psi, G=h2 * G, B=h2 * Bv, D=h2 * Dv, C=h2 * Cv)

    def _contact(self, x, project=True, derivatives=0):
        """(kappa-scaled energy, gradient, Hessian) of the self-contact pairs
        active at x: derivatives 0 energy only, 1 with the gradient, 2 with
        the gradient and the Hessian."""
        from . import selfcontact as scm
        pairs = scm.active_pairs_filtered(x, self.sc["surf"], self.sc["dhat"])
        if not derivatives:
            return self.sc["kappa"] * scm.pairs_energy(x, self.b.rest, pairs, self.sc["dhat"]), None, None
        return scm.contact_terms_sparse(x, self.b.rest, pairs, self.sc["dhat"], self.sc["kappa"], project,
                                        hessian=derivatives == 2)

    def energy(self, x):
        p = self.energy_parts(x)
        return p["K"] + p["Psi"] + p["G"] + p["B"] + p["D"] + p["C"]

    def energy_scale(self, x):
        p = self.energy_parts(x)
        return sum(abs(v) for v in p.values())

    def gradient(self, x):
        b, h2 = self.b, self.alpha * self.h * self.h
        g = b.mass[:, None] * (x - self.xtilde)
        F = b.deformation_gradient(x)
        P = snh_P(F, b.mu, b.lam)
        ge = b.vol[:, None, None] * np.einsum("tip,tap->tai", P, b.beta)  # [T,4,3]
        gel = np.zeros_like(x)
        np.add.at(gel, b.tets.ravel(), ge.reshape(-1, 3))
        g += h2 * gel
        g -= h2 * b.mass[:, None] * self.gravity[None, :]
        if self.hs is not None:
            n = np.asarray(self.hs["normal"], dtype=np.float64)
            d1 = barrier_d1(self._dist(x), float(self.hs["dhat"]))
            g += h2 * float(self.hs["kappa"]) * d1[:, None] * n[None, :]
        if self.fric is not None:
            u = (x - self.x_t) @ self.fric["P"]
            y = np.linalg.norm(u, axis=1)
            f1 = friction_f1(y, self.fric["eh"])
            c1 = np.where(y > 0, f1 / np.where(y > 0, y, 1.0), 2.0 / self.fric["eh"])  # f1(y)/y, 2/eh at 0
            g += h2 * (self.fric["mulam"] * c1)[:, None] * u
        if self.sc is not None:
            g += h2 * self._contact(x, derivatives=1)[1]
        return g

    def element_hessians(self, x, project=True):
        """12x12 elastic Hessians V_e beta^T (d2Psi/dF2) beta, [T,12,12], row (a,i)."""
        b = self.b
        F = b.deformation_gradient(x)
        C = snh_dPdF(F, b.mu, b.lam)
        if project:
            C = project_psd(C)
        # dF_ip / dx_bj = delta_ij beta_bp  ->  D [T, 9, 12] with row 3i+p, col 3b+j
        T = len(F)
        D = np.zeros((T, 3, 3, 4, 3))
        for i in range(3):
            D[:, i, :, :, i] = np.transpose(b.beta, (0, 2, 1))
        D = D.reshape(T, 9, 12)
        He = np.transpose(D, (0, 2, 1)) @ C @ D
        return b.vol[:, None, None] * He

    def hessian(self, x, project=True):
        """Sparse 3n x 3n Hessian M + h^2 (sum_e H_e + kappa b'' n n^T)."""
        b, h2 = self.b, self.alpha * self.h * self.h
        n3 = 3 * b.n
        He = h2 * self.element_hessians(x, project)
        dof = (3 * b.tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
        rows = np.repeat(dof, 12, axis=1).ravel()
        cols = np.tile(dof, (1, 12)).ravel()
        H = sp.coo_matrix((He.ravel(), (rows, cols)), shape=(n3, n3)).tocsr()
        diag = np.repeat(b.mass, 3)
        H = H + sp.diags(diag)
        if self.hs is not None:
            nrm = np.asarray(self.hs["normal"], dtype=np.float64)
            d2 = barrier_d2(self._dist(x), float(self.hs["dhat"]))
            blk = h2 * float(self.hs["kappa"]) * d2[:, None, None] * np.outer(nrm, nrm)[None]
            H = H + _block_diag3(blk)
        if self.fric is not None:
            H = H + _block_diag3(h2 * self.friction_blocks(x))
        if self.sc is not None:
            H = H + h2 * self._contact(x, project=project, derivatives=2)[2]
        return H.tocsr()

    def friction_blocks(self, x):
        """Per-vertex 3x3 Hessian of D: mu lambda [f1/y P + (f0'' - f1/y) u u^T / y^2]
        (positive semi-definite for this f0; the limit 2/eh P at rest)."""
        P, eh = self.fric["P"], self.fric["eh"]
        u = (x - self.x_t) @ P
        y = np.linalg.norm(u, axis=1)
        ys = np.where(y > 0, y, 1.0)
        c1 = np.where(y > 0, friction_f1(y, eh) / ys, 2.0 / eh)
        c2 = np.where(y > 0, (friction_f2(y, eh) - c1) / (ys * ys), 0.0)
        blk = c1[:, None, None] * P[None] + c2[:, None, None] * np.einsum("vi,vj->vij", u, u)
        return self.fric["mulam"][:, None, None] * blk


def _block_diag3(blk):
    n = len(blk)
    r = (3 * np.arange(n)[:, None, None] + np.arange(3)[None, :, None]).repeat(3, axis=2)
    c = (3 * np.arange(n)[:, None, None] + np.arange(3)[None, None, :]).repeat(3, axis=1)
    return sp.coo_matrix((blk.ravel(), (r.ravel(), c.ravel())), shape=(3 * n, 3 * n)).tocsr()
