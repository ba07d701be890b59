"""Seeded synthetic scenes shaped like the paper's workloads.

This module builds meshes, material fields, boundary conditions and initial
states only.  It holds none of the method's arithmetic (no energies, masses,
volumes or solver steps), so that both the CPU oracle and the GPU library can
take their inputs from it without sharing any part of the computation.

The paper's own meshes (Table 1) are not available; the scenes below stand in
for them with the sizes, stiffness contrasts and boundary conditions the paper
describes (Sec. 5, Tables 1-2).

Every scene is a plain dict of numpy arrays / scalars:

  rest   float64 [n,3]   reference positions (also x at t=0 unless "x0")
  tets   int32   [T,4]   positively oriented tetrahedra (by construction)
  E, nu, rho  float64 [T]
  gravity float64 [3]
  dirichlet int32 [nd]   prescribed vertices (may be empty)
  dbc_targets callable k -> float64 [nd,3] targets for step k (k = 1, 2, ...)
  halfspace None or dict(normal, offset, dhat, kappa)
  selfcontact (optional) dict(dhat, kappa): IPC contact between the mesh's
              own surface primitives
  x0, v0 float64 [n,3]
  dt float, steps int, name str
"""
from __future__ import annotations

import itertools
import math

import numpy as np

# ---------------------------------------------------------------------------
# Kuhn (Freudenthal) split of a hexahedral grid into 6 tets per cell.
# Each tet follows one permutation (a,b,c) of the axes:
#   v0 = corner, v1 = v0+e_a, v2 = v1+e_b, v3 = v2+e_c.
# Its edge matrix [e_a, e_a+e_b, e_a+e_b+e_c] has determinant sign(perm),
# so odd permutations swap v2/v3 to keep every tet positively oriented.
# The split uses the same diagonal in every cell, hence it is conforming.
# ---------------------------------------------------------------------------
_PERMS = list(itertools.permutations(range(3)))


def _perm_sign(p):
    s = 1
    p = list(p)
    for i in range(3):
        for j in range(i + 1, 3):
            if p[i] > p[j]:
                s = -s
    return s


def _kuhn_local():
    """Local corner offsets (4 corners as 3-bit ints) of the 6 Kuhn tets."""
    out = []
    for p in _PERMS:
        c = [0]
        acc = 0
        for ax in p:
            acc |= 1 << ax
            c.append(acc)
        if _perm_sign(p) < 0:
            c[2], c[3] = c[3], c[2]
        out.append(c)
    return np.array(out, dtype=np.int64)  # [6,4] bitmask offsets


def kuhn_voxels(mask: np.ndarray, h: float, origin=(0.0, 0.0, 0.0)):
    """Tetrahedralize the voxels where mask[i,j,k] is True (6 Kuhn tets each).

    Returns (rest [n,3], tets [T,4] int32, voxel_of_tet [T]); unused grid
    corners are dropped and vertices are numbered in lexicographic (k,j,i)
    order of the grid, which keeps neighbouring vertices close in memory.
    """
    nx, ny, nz = mask.shape
    vox = np.argwhere(mask)  # [V,3] (i,j,k)
    loc = _kuhn_local()  # [6,4]
    corner = np.stack([(loc >> a) & 1 for a in range(3)], axis=-1)  # [6,4,3]
    ijk = vox[:, None, None, :] + corner[None]  # [V,6,4,3]
    gid = ijk[..., 0] + (nx + 1) * (ijk[..., 1] + (ny + 1) * ijk[..., 2])
    gid = gid.reshape(-1, 4)
    used, inv = np.unique(gid, return_inverse=True)
    tets = inv.reshape(-1, 4).astype(np.int32)
    gi = used % (nx + 1)
    gj = (used // (nx + 1)) % (ny + 1)
    gk = used // ((nx + 1) * (ny + 1))
    rest = np.stack([gi, gj, gk], axis=1).astype(np.float64) * h + np.asarray(origin, dtype=np.float64)
    vox_of_tet = np.repeat(np.arange(len(vox)), 6)
    return rest, tets, vox_of_tet, vox


def kuhn_cube(N: int, size: float = 1.0):
    """Unit cube (side `size`) as N^3 hexes x 6 tets: (N+1)^3 vertices."""
    mask = np.ones((N, N, N), dtype=bool)
    rest, tets, vot, vox = kuhn_voxels(mask, size / N)
    return rest, tets, vot, vox


def _tet_barycentres(rest, tets):
    return rest[tets].mean(axis=1)


def _empty_dbc():
    return np.zeros(0, dtype=np.int32)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
GRAVITY = np.array([0.0, 0.0, -9.81])


def plain_cube(N: int = 8, seed: int = 0, e_lo: float = 1e5, e_hi: float = 1e8,
               nu: float = 0.45, rho: float = 1000.0, dt: float = 1.0 / 60.0, steps: int = 1):
    """Plain method, FP64 workload: unit cube as N^3 hexes x 6 tets (N=8: 729
    vertices, 3,072 tets), stable Neo-Hookean, per-tet Young's modulus
    log-uniform in [e_lo, e_hi] from `seed`, bottom face pinned, gravity, one
    implicit Euler step of dt = 1/60."""
    rest, tets, _, _ = kuhn_cube(N)
    rng = np.random.default_rng(seed)
    T = len(tets)
    E = np.exp(rng.uniform(math.log(e_lo), math.log(e_hi), size=T))
    dbc = np.nonzero(rest[:, 2] <= 1e-12)[0].astype(np.int32)
    tgt = rest[dbc].copy()
    return dict(name=f"plain_cube_{N}", rest=rest, tets=tets, E=E, nu=np.full(T, nu),
                rho=np.full(T, rho), gravity=GRAVITY.copy(), dirichlet=dbc,
                dbc_targets=lambda k, t=tgt: t, halfspace=None,
                x0=rest.copy(), v0=np.zeros_like(rest), dt=dt, steps=steps)


def inclusion_block(N: int = 32, seed: int = 0, n_incl: int = 20, e_soft: float = 1e5,
                    e_stiff: float = 1e10, nu: float = 0.49, rho: float = 1000.0,
                    drive: float = 0.1, ramp_steps: int = 10, steps: int = 10,
                    dt: float = 1.0 / 60.0):
    """Heterogeneous block: N^3 hexes x 6 tets (N=32: 35,937 vertices,
    196,608 tets), matrix E=e_soft with `n_incl` seeded spherical inclusions
    (centre ~U[0,1]^3, radius ~U[0.05,0.15]) at E=e_stiff; a tet is stiff when
    its barycentre lies inside an inclusion.  Bottom face pinned; the top face
    is driven down by drive/ramp_steps per step for `ramp_steps` steps, then
    held (x, y fixed).  Gravity on, dt = 1/60."""
    rest, tets, _, _ = kuhn_cube(N)
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_incl, 3))
    radii = rng.uniform(0.05, 0.15, size=n_incl)
    bc = _tet_barycentres(rest, tets)
    stiff = np.zeros(len(tets), dtype=bool)
    for c, r in zip(centres, radii):
        stiff |= ((bc - c) ** 2).sum(axis=1) < r * r
    T = len(tets)
    E = np.where(stiff, e_stiff, e_soft)
    bot = np.nonzero(rest[:, 2] <= 1e-12)[0]
    top = np.nonzero(rest[:, 2] >= 1.0 - 1e-12)[0]
    dbc = np.concatenate([bot, top]).astype(np.int32)
    base = rest[dbc].copy()
    is_top = np.concatenate([np.zeros(len(bot), bool), np.ones(len(top), bool)])

    def targets(k, base=base, is_top=is_top):
        t = base.copy()
        kk = min(k, ramp_steps)
        t[is_top, 2] -= drive * kk / ramp_steps
        return t

    return dict(name=f"inclusion_block_{N}_s{seed}", rest=rest, tets=tets, E=E,
                nu=np.full(T, nu), rho=np.full(T, rho), gravity=GRAVITY.copy(),
                dirichlet=dbc, dbc_targets=targets, halfspace=None,
                x0=rest.copy(), v0=np.zeros_like(rest), dt=dt, steps=steps,
                stiff=stiff)


def gyroid_sphere(res: int = 64, period: int = 8, thresh: float = 0.3, E: float = 1e7,
                  nu: float = 0.45, rho: float = 1000.0, speed: float = 5.0,
                  gap: float = 0.05, dhat: float = 1e-3, dt: float = 1.0 / 100.0,
                  steps: int = 100):
    """Contact scene: sphere of radius 0.5 voxelized at res^3 (voxel centre
    inside the sphere), masked by the gyroid sheet
    |sin x cos y + sin y cos z + sin z cos x| < thresh evaluated at each voxel's
    minimum corner with x = 2*pi*i/period.  The lowest vertex starts `gap`
    above a rigid slab z = 0 and the body moves down at `speed` m/s.
    res=64 gives 219,096 tets and 115,533 vertices."""
    h = 1.0 / res
    i = np.arange(res)
    I, J, K = np.meshgrid(i, i, i, indexing="ij")
    cx, cy, cz = (I + 0.5) * h - 0.5, (J + 0.5) * h - 0.5, (K + 0.5) * h - 0.5
    inside = cx * cx + cy * cy + cz * cz < 0.25
    w = 2.0 * math.pi / period
    x, y, z = w * I, w * J, w * K
    G = np.sin(x) * np.cos(y) + np.sin(y) * np.cos(z) + np.sin(z) * np.cos(x)
    mask = inside & (np.abs(G) < thresh)
    rest, tets, _, _ = kuhn_voxels(mask, h)
    rest[:, 2] += gap - rest[:, 2].min()
    T = len(tets)
    kappa = E * h  # barrier stiffness: contact modulus x voxel edge length
    v0 = np.zeros_like(rest)
    v0[:, 2] = -speed
    return dict(name=f"gyroid_sphere_{res}", rest=rest, tets=tets, E=np.full(T, E),
                nu=np.full(T, nu), rho=np.full(T, rho), gravity=GRAVITY.copy(),
                dirichlet=_empty_dbc(), dbc_targets=lambda k: np.zeros((0, 3)),
                halfspace=dict(normal=np.array([0.0, 0.0, 1.0]), offset=0.0, dhat=dhat, kappa=kappa),
                x0=rest.copy(), v0=v0, dt=dt, steps=steps)


def sliding_cube(N: int = 6, size: float = 0.2, E: float = 1e6, nu: float = 0.4, rho: float = 1000.0,
                 mu: float = 0.5, eps_v: float = 1e-3, velocity=(1.0, 0.5, 0.0), dhat: float = 1e-3,
                 dt: float = 1.0 / 100.0, steps: int = 10):
    """Friction scene: a Kuhn N^3 cube of edge `size` resting on a rigid slab
    z = 0 (bottom layer at dhat / 2, inside the barrier's range) and sliding
    with the given tangential velocity; gravity; lagged Coulomb friction
    coefficient mu with smoothing velocity eps_v.  The barrier stiffness is
    chosen so that the bottom layer's barrier forces at dhat / 2 carry the
    cube's weight (the slide starts close to vertical equilibrium)."""
    rest, tets, _, _ = kuhn_cube(N, size)
    rest = rest.copy()
    rest[:, 2] += 0.5 * dhat
    T = len(tets)
    v0 = np.tile(np.asarray(velocity, dtype=np.float64), (len(rest), 1))
    d, e = 0.5 * dhat, -0.5 * dhat
    b1 = abs(-2.0 * e * math.log(d / dhat) - e * e / d)  # |b'(dhat / 2)|
    kappa = rho * size ** 3 * abs(GRAVITY[2]) / ((N + 1) ** 2 * b1)
    return dict(name=f"sliding_cube_{N}", rest=rest, tets=tets, E=np.full(T, E), nu=np.full(T, nu),
                rho=np.full(T, rho), gravity=GRAVITY.copy(), dirichlet=_empty_dbc(),
                dbc_targets=lambda k: np.zeros((0, 3)),
                halfspace=dict(normal=np.array([0.0, 0.0, 1.0]), offset=0.0, dhat=dhat, kappa=kappa, mu=mu,
                               eps_v=eps_v),
                x0=rest.copy(), v0=v0, dt=dt, steps=steps)


def stacked_cubes(N: int = 3, size: float = 0.1, top: float = 0.08, twist_deg: float = 15.0, gap: float = 1e-3,
                  dhat: float = 2e-3, E: float = 1e5, nu: float = 0.4, rho: float = 1000.0, speed: float = 0.5,
                  dt: float = 1.0 / 100.0, steps: int = 10, free: bool = False):
    """Self-contact scene: two Kuhn N^3 cubes in one mesh.  The lower one
    (edge `size`) has its bottom face pinned; the upper one (edge `top`),
    turned by twist_deg about the vertical axis so that edges cross at an
    angle, centred a little off the lower one's centre line, starts `gap` above the lower one's
    top face and moves down at `speed` m/s under gravity.  The two bodies
    meet only through IPC self-contact (selfcontact = dict(dhat, kappa)).
    With free=True nothing is pinned, there is no gravity and the lower cube
    moves up at `speed` (a head-on collision of two free bodies)."""
    r0, t0, _, _ = kuhn_cube(N, size)
    r1, t1, _, _ = kuhn_cube(N, top)
    a = math.radians(twist_deg)
    rot = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])
    c1 = np.array([top / 2, top / 2, 0.0])
    # centred slightly off the lower cube's centre line, so that no vertex
    # of one surface lies exactly above a vertex or edge of the other
    r1 = (r1 - c1) @ rot.T + np.array([0.511 * size, 0.493 * size, size + gap])
    rest = np.concatenate([r0, r1])
    tets = np.concatenate([t0, t1 + len(r0)]).astype(np.int32)
    T = len(tets)
    v0 = np.zeros_like(rest)
    v0[len(r0):, 2] = -speed
    h = size / N
    kappa = E * h  # barrier stiffness: contact modulus x cell edge length
    if free:
        v0[:len(r0), 2] = speed
        dbc, grav = _empty_dbc(), np.zeros(3)
    else:
        dbc, grav = np.nonzero(rest[:, 2] <= 1e-12)[0].astype(np.int32), GRAVITY.copy()
    tgt = rest[dbc].copy()
    return dict(name=f"stacked_cubes_{N}", rest=rest, tets=tets, E=np.full(T, E), nu=np.full(T, nu),
                rho=np.full(T, rho), gravity=grav, dirichlet=dbc, dbc_targets=lambda k, t=tgt: t,
                halfspace=None, selfcontact=dict(dhat=dhat, kappa=kappa), n_lower=len(r0),
                x0=rest.copy(), v0=v0, dt=dt, steps=steps)


def batch_scenes(n_scenes: int = 64, seed: int = 0, t_lo: float = 1e3, t_hi: float = 5e4,
                 e_lo: float = 1e5, e_hi: float = 1e9, nu: float = 0.45, rho: float = 1000.0,
                 dt: float = 1.0 / 60.0, steps: int = 10):
    """Many independent uneven scenes: cubes or ellipsoids (p = 1/2) whose tet
    count is drawn log-uniform in [t_lo, t_hi] through the grid resolution;
    per-tet E log-uniform in [e_lo, e_hi]; bottom vertex layer pinned."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scenes):
        target = math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))
        ellip = rng.uniform() < 0.5
        if ellip:
            ax = np.array([0.5, rng.uniform(0.3, 0.5), rng.uniform(0.3, 0.5)])
            frac = math.pi / 6.0 * (2 * ax).prod()  # ellipsoid / bounding-box volume
            N = max(3, int(round((target / (6.0 * frac)) ** (1.0 / 3.0))))
            h = 1.0 / N
            c = (np.arange(N) + 0.5) * h - 0.5
            X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
            mask = (X / ax[0]) ** 2 + (Y / ax[1]) ** 2 + (Z / ax[2]) ** 2 < 1.0
            rest, tets, _, _ = kuhn_voxels(mask, h)
        else:
            N = max(2, int(round((target / 6.0) ** (1.0 / 3.0))))
            rest, tets, _, _ = kuhn_cube(N)
        T = len(tets)
        E = np.exp(rng.uniform(math.log(e_lo), math.log(e_hi), size=T))
        zmin = rest[:, 2].min()
        dbc = np.nonzero(rest[:, 2] <= zmin + 1e-12)[0].astype(np.int32)
        tgt = rest[dbc].copy()
        out.append(dict(name=f"batch_{seed}_{s}", rest=rest, tets=tets, E=E, nu=np.full(T, nu),
                        rho=np.full(T, rho), gravity=GRAVITY.copy(), dirichlet=dbc,
                        dbc_targets=lambda k, t=tgt: t, halfspace=None, x0=rest.copy(),
                        v0=np.zeros_like(rest), dt=dt, steps=steps))
    return out


def learned_trajectory_scene(seed: int, N: int = 32, steps: int = 60):
    """Warm-start training / evaluation trajectories: the heterogeneous-block
    generator with a 10-step ramp followed by `steps - 10` held steps."""
    return inclusion_block(N=N, seed=seed, steps=steps, ramp_steps=10)


def learned_drive_scene(seed: int, N: int = 32, steps: int = 60, geometry_seed: int = 0):
    """Warm-start trajectories on one fixed heterogeneous block (inclusions
    from geometry_seed) whose drive varies with `seed`: the top face moves
    down by an amplitude ~U[0.05, 0.15] m over a ramp of ~U{6..14} steps, then
    is held.  One geometry keeps the coarse coordinates of a material-aware
    basis meaningful across trajectories."""
    rng = np.random.default_rng(seed)
    drive = float(rng.uniform(0.05, 0.15))
    ramp = int(rng.integers(6, 15))
    s = inclusion_block(N=N, seed=geometry_seed, steps=steps, drive=drive, ramp_steps=ramp)
    s["name"] = f"inclusion_block_{N}_g{geometry_seed}_drive{seed}"
    return s


TRAIN_SEEDS = list(range(1000, 1200))
HELDOUT_SEEDS = list(range(2000, 2020))


def spd_bsr_pattern(N: int, seed: int = 0, permute: bool = False):
    """Kuhn-grid vertex adjacency (block pattern of a BSR3 matrix) with values
    ~N(0,1) and a dominant diagonal block, for SpMV measurements at sizes
    beyond the simulation workloads.  Returns (row_ptr, col, vals[nnzb,3,3])."""
    rest, tets, _, _ = kuhn_cube(N)
    n = len(rest)
    a = tets[:, [0, 0, 0, 1, 1, 2]].ravel().astype(np.int64)
    b = tets[:, [1, 2, 3, 2, 3, 3]].ravel().astype(np.int64)
    if permute:
        p = np.random.default_rng(seed + 1).permutation(n)
        a, b = p[a], p[b]
    key = np.unique(np.concatenate([np.minimum(a, b) * n + np.maximum(a, b)]))
    i, j = key // n, key % n
    rows = np.concatenate([np.arange(n), i, j])
    cols = np.concatenate([np.arange(n), j, i])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    rng = np.random.default_rng(seed)
    vals = rng.standard_normal((len(rows), 3, 3))
    diag = rows == cols
    vals[diag] += 40.0 * np.eye(3)
    return row_ptr, cols.astype(np.int32), vals


def mlp_init(in_dim: int, width: int, out_dim: int, seed: int = 0):
    """Seeded initial weights of the warm-start network (uniform in
    +-1/sqrt(fan_in), row-major [out][in]) as float32, shared by the GPU
    trainer and the oracle."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, (o, i) in (("0", (width, in_dim)), ("1", (width, width)), ("2", (out_dim, width))):
        bound = 1.0 / math.sqrt(i)
        out["W" + name] = rng.uniform(-bound, bound, size=(o, i)).astype(np.float32)
        out["b" + name] = rng.uniform(-bound, bound, size=o).astype(np.float32)
    return out


def minibatch_order(n_samples: int, batch: int, n_steps: int, seed: int = 0):
    """Sample indices of every training step (a fresh permutation per epoch),
    shape [n_steps, batch], int32."""
    rng = np.random.default_rng(seed)
    idx = []
    while len(idx) < n_steps * batch:
        idx.extend(rng.permutation(n_samples).tolist())
    return np.asarray(idx[:n_steps * batch], dtype=np.int32).reshape(n_steps, batch)


def vertex_order(rest: np.ndarray, tets: np.ndarray, kind: str, seed: int = 0) -> np.ndarray:
    """A vertex numbering for SpMV measurements: 'natural' (the generator's),
    'random' (a seeded permutation, the unstructured-mesh stand-in) or 'rcm'
    (reverse Cuthill-McKee on the tet edge graph).  Returns perm with new
    vertex i = old vertex perm[i]."""
    n = len(rest)
    if kind == "natural":
        return np.arange(n)
    if kind == "random":
        return np.random.default_rng(seed).permutation(n)
    if kind == "rcm":
        import scipy.sparse as sp
        from scipy.sparse.csgraph import reverse_cuthill_mckee
        a = tets[:, [0, 0, 0, 1, 1, 2]].ravel()
        b = tets[:, [1, 2, 3, 2, 3, 3]].ravel()
        A = sp.coo_matrix((np.ones(len(a)), (a, b)), shape=(n, n))
        A = (A + A.T).tocsr()
        return np.asarray(reverse_cuthill_mckee(A, symmetric_mode=True))
    raise ValueError(kind)


def permute_vertices(s: dict, perm: np.ndarray) -> dict:
    """The same scene with its vertices renumbered (new vertex i = old vertex
    perm[i]); Dirichlet targets keep the order of the Dirichlet list."""
    perm = np.asarray(perm)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    out = dict(s)
    out["rest"] = s["rest"][perm]
    out["x0"] = s["x0"][perm]
    out["v0"] = s["v0"][perm]
    out["tets"] = inv[s["tets"]].astype(np.int32)
    out["dirichlet"] = inv[s["dirichlet"]].astype(np.int32)
    return out

