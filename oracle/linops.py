"""Plain definitions of the linear operators on the hot path (FP64 oracle).

Test infrastructure only.  Each function is the textbook definition, written
with library primitives (scipy.sparse products, numpy dense algebra):

  bsr_matvec        y = H x for a 3x3 block-sparse matrix (the Newton
                    system H d = -g, Sec. 3.1)
  dense_basis       the stacked 3x12 blocks phi_i(x) P_i(x - x_i) of the
                    linear-blend-skinning basis (Eq. LBS, Sec. 3.4), as an
                    explicit 3n x 12m matrix; P_i = I_3 (x) [1, dx, dy, dz]
  restrict/prolong  U^T r and U q (the matrix-free triple product of
                    Sec. 3.7.1: lift, apply H, restrict)
  galerkin          U^T H U, the subspace Hessian
  coarse_solve      (U^T H U)^{-1} c by Cholesky
  block_jacobi_inverse  inverses of the 3x3 diagonal blocks
Parity status: pinned through tests/test_oracle_linops.py against brute force
(explicit loops over blocks and vertices).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def bsr_matrix(row_ptr, col, vals, n):
    return sp.bsr_matrix((np.asarray(vals, dtype=np.float64).reshape(-1, 3, 3), np.asarray(col),
                          np.asarray(row_ptr)), shape=(3 * n, 3 * n))


def bsr_matvec(row_ptr, col, vals, x):
    n = len(row_ptr) - 1
    return (bsr_matrix(row_ptr, col, vals, n) @ np.asarray(x, dtype=np.float64).ravel()).reshape(-1, 3)


def dense_basis(rest, origins, vptr, vhandle, vphi, m):
    """Explicit U (3n x 12m): row block v, column block i holds
    phi_vi * (I_3 (x) [1, x_v - o_i])."""
    n = len(rest)
    U = np.zeros((3 * n, 12 * m))
    for v in range(n):
        for k in range(vptr[v], vptr[v + 1]):
            i = int(vhandle[k])
            p = np.concatenate([[1.0], rest[v] - origins[i]])
            for a in range(3):
                U[3 * v + a, 12 * i + 4 * a:12 * i + 4 * a + 4] += vphi[k] * p
    return U


def restrict(U, r):
    return U.T @ np.asarray(r, dtype=np.float64).ravel()


def prolong(U, e):
    return (U @ np.asarray(e, dtype=np.float64)).reshape(-1, 3)


def galerkin(U, H):
    Hd = H.toarray() if sp.issparse(H) else np.asarray(H)
    return U.T @ Hd @ U


def coarse_solve(A, c):
    L = np.linalg.cholesky(A)
    y = sla.solve_triangular(L, c, lower=True)
    return sla.solve_triangular(L.T, y, lower=False)


def block_jacobi_inverse(row_ptr, col, vals, n):
    """Inverse of each 3x3 diagonal block."""
    vals = np.asarray(vals, dtype=np.float64).reshape(-1, 3, 3)
    out = np.zeros((n, 3, 3))
    for i in range(n):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            if col[k] == i:
                out[i] = np.linalg.inv(vals[k])
    return out
