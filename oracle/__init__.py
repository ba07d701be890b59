"""CPU oracle for the multilevel elastodynamics hot path (test infrastructure).

This package is a plain, slow, FP64 implementation of what the GPU library
computes.  It exists only to check the GPU path: the tests, the smoke check
and the benchmark's CPU-baseline leg may use it; the library never does.  It
shares no code with the GPU library; both take inputs from the `scenes`
generators only.

Modules
  fem       incremental potential of Eq. (IP) with implicit Euler (Sec. 3.1):
            stable Neo-Hookean elasticity, lumped inertia, gravity, IPC
            half-space barrier; energies, gradients, PSD-projected Hessians
  newton    full-space Newton with a sparse direct solve, CCD-filtered
            backtracking line search (Sec. 3.1 Newton step, Sec. 3.9)
  linops    plain definitions of the linear operators on the hot path:
            BSR3 products, basis restriction / prolongation (Eq. LBS),
            Galerkin coarse operator, coarse Cholesky solves
  basis     sparse material-aware basis weights given a partitioning
            (Sec. 3.5: local stiffness-weighted biharmonic solves, clipping,
            partition of unity, Dirichlet-compatible variant)
  mlp       FP64 forward / backward / Adam of the warm-start network
  paper     the paper's three-level inexact Newton solve (Alg. 1 and 2)
  cubature  modal moment-fitting cubature of the subspace Hessian (Alg. 3)
  selfcontact  IPC point-triangle / edge-edge barriers between surface
            primitives and their time of impact under linear motion

Parity status of each function is stated in its module header.
"""
