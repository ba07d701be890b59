/*
 * ms.h -- C ABI of the MI355X multilevel elastodynamics timestep library.
 *
 * The library advances a tetrahedral mesh by implicit Euler timesteps,
 * x^{t+1} = argmin_x E(x) with the incremental potential of Eq. (IP)
 * (Sec. 3.1): E = 1/2 ||x - x~||_M^2 + h^2 (Psi + B), x~ = x^t + h v^t,
 * v^{t+1} = (x^{t+1} - x^t) / h.  Each timestep is a Newton solve
 * (H d = -g, Sec. 3.1) whose linear systems are solved by preconditioned
 * conjugate gradient; the preconditioner is either 3x3 block-Jacobi or the
 * two-level preconditioner built from the sparse material-aware basis U of
 * Sec. 3.4-3.6 (restriction U^T r, a dense Cholesky solve with U^T H U,
 * prolongation U e).  The paper's own three-level inexact Newton solve
 * (Alg. 1 and 2) is available as a mode.
 *
 * Conventions for every call below:
 *   - All functions return ms_status; MS_OK (0) is success.  On failure the
 *     context keeps a message retrievable with ms_last_error().
 *   - Unless stated otherwise, array arguments are HOST pointers that are
 *     read (or written) during the call only; the caller keeps ownership.
 *     Vectors of points are row-major [n][3] doubles.
 *   - Device memory is obtained through ms_device.alloc (for instance a
 *     PyTorch caching allocator) or hipMalloc when alloc is NULL, and all
 *     device work is enqueued on ms_device.hip_stream.  A context owns every
 *     device buffer it allocates and releases it in ms_destroy().
 *   - A context may be used by one host thread at a time.
 *   - Call order: ms_create -> ms_upload_mesh -> ms_upload_material ->
 *     (ms_set_gravity, ms_set_dirichlet, ms_add_halfspace in any order) ->
 *     ms_set_state -> (ms_build_basis | ms_set_basis, optional) -> ms_step*.
 *     A call made before its prerequisites returns MS_E_ORDER.
 */
#ifndef MS_H
#define MS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ms_ctx ms_ctx;

typedef enum {
  MS_OK = 0,
  MS_E_ARG = -1,        /* invalid argument (null pointer, size, index out of range) */
  MS_E_MESH = -2,       /* degenerate or inverted rest tetrahedron                    */
  MS_E_ORDER = -3,      /* call made before its prerequisites                          */
  MS_E_DEVICE = -4,     /* a HIP call failed                                           */
  MS_E_NOMEM = -5,      /* device allocation failed                                    */
  MS_E_NOCONV = -6,     /* Newton did not converge in max_newton iterations            */
  MS_E_LINESEARCH = -7, /* no energy decrease within the backtracking budget          */
  MS_E_NONFINITE = -8   /* NaN or Inf in an input or in the iterate                    */
} ms_status;

/* Device, stream and allocator the context runs on.  alloc/free may be NULL
 * (then hipMalloc/hipFree are used).  hip_stream is a hipStream_t (NULL =
 * the null stream). */
typedef struct {
  int device;
  void* hip_stream;
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} ms_device;

typedef enum { MS_PREC_FP64 = 0, MS_PREC_MIXED = 1 } ms_precision;
/* Preconditioners of the plain path.  S = 3x3 block-Jacobi of H,
 * Q = U (U^T H U)^-1 U^T the coarse correction on the basis U:
 *   MS_PC_BLOCK_JACOBI         z = S r
 *   MS_PC_TWO_LEVEL            z = S r + Q (r - H S r)   (smoothing then coarse
 *                              correction; PCG starts from d_0 = Q(-g), which
 *                              makes the iteration a deflated / balancing
 *                              two-level method)
 *   MS_PC_TWO_LEVEL_ADDITIVE   z = S r + Q r
 *   MS_PC_TWO_LEVEL_VCYCLE     symmetric V(1,1): z1 = L r, z2 = z1 + Q (r - H z1),
 *                              z = z2 + L (r - H z2), with L the l1-scaled 3x3
 *                              block-Jacobi inverse (diagonal block of H plus, on
 *                              its diagonal, the absolute row sums of the row's
 *                              other blocks at free vertices), which keeps the
 *                              V-cycle SPD for any SPD coarse matrix */
typedef enum {
  MS_PC_BLOCK_JACOBI = 0,
  MS_PC_TWO_LEVEL = 1,
  MS_PC_TWO_LEVEL_ADDITIVE = 2,
  MS_PC_TWO_LEVEL_VCYCLE = 3
} ms_preconditioner;
typedef enum { MS_MODE_PLAIN = 0, MS_MODE_PAPER = 1 } ms_mode;
/* How the coarse (subspace) matrix U^T H U is integrated (Sec. 3.8):
 *   MS_COARSE_EXACT      every tet's elastic Hessian (the Galerkin product)
 *   MS_COARSE_CUBATURE   the elastic part from the installed cubature only,
 *                        h^2 sum_q (w_q / V_q) U_q^T H_q U_q; inertia, barrier
 *                        and friction curvature stay exact.  Symmetric
 *                        positive semi-definite for non-negative weights.
 *                        Used by the additive and V-cycle preconditioners
 *                        and paper mode; ms_step and ms_apply_preconditioner
 *                        reject MS_PC_TWO_LEVEL (its deflation needs the
 *                        exact matrix) with MS_E_ARG. */
typedef enum { MS_COARSE_EXACT = 0, MS_COARSE_CUBATURE = 1 } ms_coarse_integration;

/* Parameters of one timestep solve.  ms_solver_defaults() fills them. */
typedef struct {
  int32_t mode;            /* ms_mode                                                   */
  int32_t precision;       /* ms_precision: FP64, or FP32 Hessian/SpMV/preconditioner
                              with FP64 gradient, residual replacement and line search */
  int32_t preconditioner;  /* ms_preconditioner (plain mode)                            */
  int32_t max_newton;      /* Newton iteration cap (MS_E_NOCONV beyond it)              */
  int32_t max_pcg;         /* PCG iteration cap per Newton iteration                   */
  double newton_tol;       /* plain mode: stop when a full step has
                              ||d||_2 <= newton_tol * max(||x - x^t||_2, abs_floor),
                              or ||d||_2 <= 1e-13 ||x||_2 (below the resolution of the
                              FP64 positions: an almost static step)                   */
  double abs_floor;        /* absolute displacement floor of that test (m)              */
  double pcg_eta_max;      /* upper bound of the PCG forcing term (see forcing)         */
  double pcg_eta_min;      /* lower bound of the forcing term                           */
  int32_t max_backtracks;  /* line-search halvings before MS_E_LINESEARCH               */
  int32_t exact_endgame;   /* 1: drop the PSD projection once steps are small           */
  int32_t warm_start;      /* 1: use the learned coarse warm start if one is set        */
  /* paper mode (Alg. 1 and 2) */
  double paper_eps;        /* termination on mean per-vertex ||d_s,v|| / h  (m/s)       */
  double subspace_rtol;    /* relative residual ||r_k|| <= subspace_rtol ||r_0|| at which the
                              affine and sparse subspace PCG solves stop (Sec. 3.7.1;
                              12x12 block-Jacobi, at most max_pcg iterations), in [0,1) */
  int32_t refine_iters;    /* fixed Jacobi-PCG iterations of the full-space refinement;
                              0: 20 or 40 from the partitions' mean hop diameter      */
  int32_t lag_window;      /* step sizes averaged by the Hessian-lag trigger             */
  double lag_threshold;    /* refresh the lagged elastic Hessian below this average     */
  int32_t lag_min_gap;     /* at most one refresh every lag_min_gap iterations          */
  /* plain mode, continued */
  int32_t forcing;         /* 0: eta = sqrt(||g||/||g_0||); 1: Eisenstat-Walker choice 2,
                              eta_k = 0.9 (||g_k||/||g_k-1||)^2 with safeguard          */
  double endgame_ratio;    /* exact (unprojected) Hessian once ||d|| <= ratio * ||x - x^t|| */
  int32_t coarse_every;    /* additive and V-cycle two-level: rebuild U^T H U and its
                              factor at the first Newton iteration of a step and then
                              every coarse_every iterations (0: once per step; the
                              preconditioner may lag H).  The smoothed form rebuilds
                              at every iteration.                                      */
  int32_t predictor;       /* initial Newton iterate: 0 x^t; 1 the inertial predictor
                              x^t + h v^t (truncated by the contact filter, Dirichlet
                              vertices at their targets), kept only if it lowers E     */
  int32_t time_kernels;    /* 1: bracket every PCG product launch of this step with HIP
                              events (PCG runs without graphs); ms_time_kernel with
                              reps = 0 then reports their average duration             */
  double coarse_move;      /* > 0, additive / V-cycle: after the first Newton iteration,
                              rebuild U^T H U and its factor only once the iterate has
                              moved by more than coarse_move * max(||x - x^t||,
                              abs_floor) since the last rebuild (replaces coarse_every) */
  int32_t mixed_max_newton; /* mixed precision: continue the timestep in FP64 after this
                              many Newton iterations without convergence (0: never)    */
  int32_t mixed_endgame_fp64; /* mixed precision: 1 = assemble and solve in FP64 once
                              ||d|| <= endgame_ratio * ||x - x^t|| (the tight solves)   */
  int32_t integrator;      /* plain mode: 0 implicit Euler; 1 BDF2 (Sec. 3.1):
                              x~ = 4/3 x^t - 1/3 x^{t-1} + h (8 v^t - 2 v^{t-1}) / 9,
                              weight 4/9 on the h^2 terms, v^{t+1} = (3 x^{t+1} - 4 x^t
                              + x^{t-1}) / (2h), using the previous plain step of this
                              context (implicit Euler when there is none: the first
                              step after ms_set_state)                               */
  int32_t projection;      /* plain mode, projected element Hessians: 0 negative
                              eigenvalues of d2Psi/dF2 clamped to zero; 1 replaced by
                              their absolute values (both positive semi-definite; the
                              minimiser does not depend on the choice)               */
  int32_t smoother;        /* plain mode, block-Jacobi or additive two-level PCG, no
                              self-contact: the block part of the preconditioner.
                              0: inverses of the 3x3 vertex blocks of H (block-Jacobi,
                              as the paper's subspace solves use per handle, Sec.
                              3.7.1); 1: exact inverses of the 24 x 24 diagonal
                              blocks of H over vertex aggregates of at most 8 (rest
                              positions binned into cubes of twice the shortest edge:
                              2 x 2 x 2 vertices on a regular grid), formed in FP64
                              each Newton iteration and applied in the Hessian's
                              precision.  MS_E_ARG otherwise; batched steps take 0    */
} ms_solver_params;

/* Statistics of the last ms_step. */
typedef struct {
  int32_t newton_iters;
  int32_t pcg_iters;          /* total over the step                                    */
  int32_t max_pcg_iters;      /* largest single solve                                   */
  int32_t backtracks;         /* total line-search halvings                             */
  int32_t hessian_refreshes;  /* paper mode: lagged-Hessian recomputations; plain mode
                                 with a basis: rebuilds of U^T H U and its factor      */
  int32_t warm_start_used;    /* 1 if the learned prediction was accepted               */
  int32_t precision_escalations; /* mixed precision: 1 if the step was continued in FP64
                                    after mixed_max_newton iterations                    */
  int32_t pcg_iters_fp64;     /* plain mode: PCG iterations run with the FP64 Hessian     */
  int32_t pcg_solves_fp64;    /* plain mode: PCG solves run with the FP64 Hessian         */
  double energy;              /* E at x^{t+1}                                            */
  double last_dnorm;          /* ||d||_2 of the last Newton step                         */
  double disp_norm;           /* ||x^{t+1} - x^t||_2                                     */
  double min_alpha;           /* smallest accepted line-search step                      */
  double time_ms;             /* host wall time of the step                              */
  int32_t subspace_pcg_iters; /* paper mode: PCG iterations of the affine and sparse
                                 subspace solves, total over the step                   */
  int32_t refine_iters;       /* paper mode: refinement CG iterations per Newton iteration
                                 (refine_iters, or 20/40 from the hop diameters)         */
  double pcg_ms;              /* plain mode: host wall time inside the PCG solves (graph
                                 replays, launch gaps and the looks at the done flag
                                 included)                                               */
} ms_step_stats;

/* Parameters of the basis construction (Sec. 3.5-3.6).  ms_basis_defaults()
 * fills them. */
typedef struct {
  int32_t n_handles;       /* target number of partitions / handles m               */
  double oversample;       /* K-means starts with ceil(oversample * m) seeds          */
  double jump_penalty;     /* stiffness factor on tets at material jumps (x softest)  */
  double prune_ratio;      /* prune when median volume > prune_ratio * own volume    */
  int32_t prune_every;     /* Lloyd iterations between pruning rounds                */
  int32_t prune_n;         /* clusters removed per pruning round                     */
  int32_t max_lloyd;       /* Lloyd iteration cap                                    */
  int32_t lattice_seeding; /* 1: seeds on a fixed lattice, no pruning (stable handle
                              indices across meshes of the same shape)              */
  uint64_t seed;
  int32_t n_threads;       /* host threads (0 = hardware concurrency)                */
  int32_t gpu_min_unknowns; /* ms_build_basis: local solves with at least this many
                               unknowns run as dense Cholesky on the GPU (0 = none;
                               default 4096); ms_basis_compute solves on the host */
  double rigid_contrast;   /* > 0: on every connected set of tets with E >=
                              rigid_contrast x min E (tets sharing a vertex are
                              connected) the weights of the free vertices are replaced
                              by their average over the set, so each handle moves the
                              set affinely (the stiff limit of the material-aware
                              weights; partition of unity kept); 0 = off (default) */
} ms_basis_params;

void ms_solver_defaults(ms_solver_params* p);
void ms_basis_defaults(ms_basis_params* p);

/* Create a context on dev->device.  *out receives the context.
 * Errors: MS_E_ARG (null), MS_E_DEVICE (device cannot be selected). */
ms_status ms_create(const ms_device* dev, ms_ctx** out);

/* Upload the reference mesh (Sec. 3.1: positions at n vertices, a simplicial
 * tet mesh).  rest_xyz [n][3], tets [T][4] vertex indices with positive
 * orientation (det[x1-x0, x2-x0, x3-x0] > 0).  Builds the block-sparse
 * Hessian pattern and the atomic-free assembly maps.
 * Errors: MS_E_ARG (index out of range, n or T < 1), MS_E_MESH (a rest tet
 * with non-positive volume), MS_E_NONFINITE. */
ms_status ms_upload_mesh(ms_ctx* c, int64_t n_verts, const double* rest_xyz, int64_t n_tets,
                         const int32_t* tets);

/* Per-tet Young's modulus E (Pa, > 0), Poisson ratio nu (in (-1, 0.5)) and
 * density rho (kg/m^3, > 0), each [T].  The elastic energy is the stable
 * Neo-Hookean density with mu = E/(2(1+nu)), lam' = E nu/((1+nu)(1-2nu)) + mu;
 * masses are lumped, m_v = sum rho V / 4.  Errors: MS_E_ARG, MS_E_ORDER. */
ms_status ms_upload_material(ms_ctx* c, const double* E, const double* nu, const double* rho);

/* Gravity g[3] (m/s^2), entering E as -h^2 sum_v m_v g . x_v. */
ms_status ms_set_gravity(ms_ctx* c, const double g[3]);

/* Dirichlet conditions (Sec. 3.5.1): vertices verts[n] are set to
 * target_xyz [n][3] at the start of every following step and their DOFs are
 * eliminated.  May be called between steps (moving targets) with the same
 * or a different vertex set (a different set invalidates a built basis:
 * build it again).  n = 0 clears them.  Errors: MS_E_ARG, MS_E_ORDER. */
ms_status ms_set_dirichlet(ms_ctx* c, int64_t n, const int32_t* verts, const double* target_xyz);

/* A rigid half-space {y : normal . y >= offset} in contact with every
 * vertex of positive lumped mass (a vertex of no tet carries no contact)
 * through the IPC log barrier b(d) = -(d - dhat)^2 ln(d/dhat) on
 * d = normal . x - offset (Eq. IP, term B), scaled by kappa (N/m).  The line
 * search keeps every vertex strictly inside the half-space.  normal need not
 * be unit length (it is normalised).  At most one half-space. */
ms_status ms_add_halfspace(ms_ctx* c, const double normal[3], double offset, double dhat, double kappa);

/* Lagged Coulomb friction against the half-space (the D term of the
 * incremental potential, Sec. 3.1; IPC's smoothed form): per vertex
 * mu lambda_v f0(|P (x_v - x_v^t)|) with P the tangent projector of the
 * plane, lambda_v = kappa |b'(d_v(x^t))| the barrier's normal force at the
 * start of the step and f0 the C1 smoothing of |u| below eps_v h (eps_v in
 * m/s).  mu = 0 turns friction off.  Plain mode only (paper mode returns
 * MS_E_ARG).  Errors: MS_E_ORDER without a half-space, MS_E_ARG for
 * mu < 0 or eps_v <= 0. */
ms_status ms_set_friction(ms_ctx* c, double mu, double eps_v);

/* IPC self-contact between the mesh's own surface primitives (Sec. 4; the
 * paper's contact model and its CCD-filtered line search, Sec. 3.9): every
 * point-triangle pair (surface vertex, surface triangle not containing it)
 * and edge-edge pair (surface edges sharing no vertex) closer than dhat adds
 * kappa b(d) to the h^2-weighted terms of Eq. IP, with b the log barrier of
 * ms_add_halfspace in the unsigned distance d between the closed primitives,
 * times IPC's mollifier of nearly parallel edges for edge-edge pairs (eps_x
 * = 1e-3 |A1 - A0|^2 |B1 - B0|^2 at rest).  The surface is the set of tet
 * faces that belong to one tet only.  Every search direction is truncated
 * by additive CCD (gap fraction 0.1) of the pairs whose swept boxes meet.
 * The constraint set is recomputed at every assembly and energy
 * evaluation; its curvature enters the Hessian in the Gauss-Newton form
 * kappa h^2 m b''(d) grad d grad d^T (positive semi-definite; the minimiser
 * is that of the exact energy).  Each surface vertex reserves `slots`
 * Hessian blocks for couplings outside its mesh neighbourhood; an assembly
 * that needs more fails with MS_E_ARG.  The two-level preconditioners'
 * coarse matrix omits the self-contact terms.  Plain mode only (not paper
 * mode, not the smoothed two-level preconditioner, not batched steps).
 * The state must be free of intersections.  Call between ms_upload_mesh and
 * ms_upload_material.  Errors: MS_E_ORDER, MS_E_ARG (dhat or kappa not
 * positive, slots outside [1, 64]). */
ms_status ms_set_self_contact(ms_ctx* c, double dhat, double kappa, int32_t slots);

/* Set positions x [n][3] and velocities v [n][3].  With a half-space every
 * vertex must lie strictly inside it.  Errors: MS_E_NONFINITE, MS_E_ARG. */
ms_status ms_set_state(ms_ctx* c, const double* x, const double* v);
ms_status ms_get_state(const ms_ctx* c, double* x, double* v);

/* Build the sparse geometry- and material-aware basis (Sec. 3.4-3.6) on the
 * host: K-means partitioning on stiffness-weighted graph geodesics (Dijkstra
 * over mesh edges whose lengths are scaled by the local stiffness; the paper
 * computes its geodesics by the heat method, Sec. 3.6.1) with the jump
 * penalty and pruning, local stiffness-weighted biharmonic solves on each
 * partition's face-neighbour subdomain, clipping, partition of unity, and
 * the Dirichlet-compatible variant when Dirichlet vertices exist.  Local
 * solves with at least p->gpu_min_unknowns unknowns run as a dense blocked
 * Cholesky on the GPU (the rest on host threads meanwhile).  Uploads
 * the basis for the two-level preconditioner and paper mode.
 * Errors: MS_E_ORDER (no mesh/material), MS_E_ARG. */
ms_status ms_build_basis(ms_ctx* c, const ms_basis_params* p);

/* The last ms_build_basis: how many local solves ran on the GPU (dense
 * Cholesky, p->gpu_min_unknowns) and its host wall time in seconds (either
 * pointer may be NULL). */
ms_status ms_get_basis_stats(const ms_ctx* c, int32_t* gpu_solves, double* seconds);

/* Install an externally computed basis: m handles with origins [m][3]; for
 * each vertex v the handles vhandle[vptr[v] .. vptr[v+1]) with weights vphi
 * (the phi_i(x_v) of Eq. LBS).  nnz = vptr[n]. */
ms_status ms_set_basis(ms_ctx* c, int32_t m, const double* origins, const int64_t* vptr,
                       const int32_t* vhandle, const double* vphi);

/* Query the installed basis: *m, *nnz; then, if the arrays are non-null,
 * origins [m][3], vptr [n+1], vhandle [nnz], vphi [nnz], and part [T] (the
 * partition of every tet, or -1 for a basis set by ms_set_basis). */
ms_status ms_get_basis_size(const ms_ctx* c, int32_t* m, int64_t* nnz);
ms_status ms_get_basis(const ms_ctx* c, double* origins, int64_t* vptr, int32_t* vhandle, double* vphi,
                       int32_t* part);

/* Host-only basis construction (no device involved): the same algorithm as
 * ms_build_basis on a mesh rest_xyz [n][3] / tets [T][4], Young's moduli
 * E [T] and Dirichlet vertices dbc [n_dbc].  *out receives an opaque result
 * that ms_basis_get queries (first with null arrays for *m and *nnz, then
 * with arrays sized origins [m][3], vptr [n+1], vhandle [nnz], vphi [nnz],
 * part [T]) and ms_basis_free releases.  The arrays can be passed to
 * ms_set_basis.  Errors: MS_E_ARG, MS_E_MESH. */
typedef struct ms_basis ms_basis;
ms_status ms_basis_compute(int64_t n, const double* rest_xyz, int64_t T, const int32_t* tets, const double* E,
                           int64_t n_dbc, const int32_t* dbc, const ms_basis_params* p, ms_basis** out);
ms_status ms_basis_get(const ms_basis* b, int32_t* m, int64_t* nnz, double* origins, int64_t* vptr,
                       int32_t* vhandle, double* vphi, int32_t* part);
void ms_basis_free(ms_basis* b);

/* Vertex aggregates of the aggregate block-Jacobi smoother (the `smoother`
 * = 1 solver option), host-only: the rule ms_step applies to a context's
 * mesh.  rest_xyz [n][3]; the vertex graph as CSR (row_ptr [n+1] from 0,
 * col [row_ptr[n]], entries 0..n-1, self entries allowed).  Positions are binned
 * into cubes of twice the graph's shortest edge, offset by half an edge (a
 * regular grid gives 2 x 2 x 2 vertices), bins ordered by (z, y, x) and
 * each split in vertex order into groups of at most 8.  *n_agg receives the
 * aggregate count; vert (caller-owned, cap entries; cap = 0 and vert = NULL
 * to query) receives 8 entries per aggregate, vertex ids padded with -1,
 * the first cap of them.  MS_E_ARG on null pointers or n < 1,
 * MS_E_NONFINITE on a non-finite position, MS_E_MESH on a malformed graph. */
ms_status ms_aggregates_compute(int64_t n, const double* rest_xyz, const int32_t* row_ptr, const int32_t* col,
                                int64_t cap, int32_t* vert, int64_t* n_agg);

/* Modal moment-fitting cubature (Sec. 3.8, modal moment fitting and its
 * solver; Alg. 3), host-only (no device involved).  Per partition p
 * (tets with part[t] == p, part [T] >= 0): the basis functions touching p,
 * evaluated per tet as the mean of their vertex weights, give the degree-2
 * moment conditions (1, u_i, u_i u_j for i <= j) with targets the
 * volume-weighted sums over all of p's tets.  Starting from n_init tets
 * drawn uniformly, non-negative least squares is solved on the drawn tets;
 * while the relative residual exceeds tol and rounds remain (at most
 * max_rounds), n_add more tets are drawn with probability proportional to
 * (A_k^T r)^2.  Draws use SplitMix64 as a counter-based generator of `seed`
 * (draw j of partition p: state seed + (2^32 p + j + 1) * 0x9E3779B97F4A7C15).
 * The basis is given as in ms_set_basis (vptr [n+1], vhandle / vphi
 * [vptr[n]], handles < m).  n_threads <= 0 uses every hardware thread.
 * *out receives an opaque result that ms_cubature_get queries (first with
 * null arrays for *n_pts, then with tets / weights of n_pts entries: the
 * selected tets ascending and their weights in volume units) and
 * ms_cubature_free releases.  Errors: MS_E_ARG. */
typedef struct ms_cubature ms_cubature;
ms_status ms_cubature_compute(int64_t n, const double* rest_xyz, int64_t T, const int32_t* tets,
                              const int32_t* part, int32_t m, const int64_t* vptr, const int32_t* vhandle,
                              const double* vphi, double tol, int32_t n_init, int32_t n_add, int32_t max_rounds,
                              uint64_t seed, int32_t n_threads, ms_cubature** out);
ms_status ms_cubature_get(const ms_cubature* q, int64_t* n_pts, int32_t* tets, double* weights,
                          double* max_rel_residual);
void ms_cubature_free(ms_cubature* q);

/* The same fit on the context's mesh and installed basis (which must carry
 * its partitioning, i.e. come from ms_build_basis), installed as by
 * ms_set_cubature.  max_rel_residual (may be NULL) receives the largest
 * relative moment residual over the partitions.  Errors: MS_E_ORDER (no
 * basis or no partitioning), MS_E_ARG. */
ms_status ms_build_cubature(ms_ctx* c, double tol, int32_t n_init, int32_t n_add, int32_t max_rounds,
                            uint64_t seed, double* max_rel_residual);

/* Install a cubature: n_pts distinct tets [n_pts] with weights >= 0 in
 * volume units (copied).  n_pts = 0 removes it (and selects
 * MS_COARSE_EXACT).  Errors: MS_E_ORDER (no mesh), MS_E_ARG (a tet out of
 * range or repeated, a negative or non-finite weight). */
ms_status ms_set_cubature(ms_ctx* c, int64_t n_pts, const int32_t* tets, const double* weights);

/* Query the installed cubature: *n_pts, then, if non-null, tets [n_pts]
 * (ascending) and weights [n_pts]. */
ms_status ms_get_cubature(const ms_ctx* c, int64_t* n_pts, int32_t* tets, double* weights);

/* Continuous collision detection of IPC self-contact primitive pairs (the
 * paper filters every search direction with additive CCD: Sec. 3.9 line
 * search, Sec. 4), on the GPU without a context.  Pair q is a point and a
 * triangle (kind[q] = 0; x12 [q][12] = point, then the triangle's three
 * vertices) or two edges (kind[q] = 1; first edge's two vertices, then the
 * second's), moving by p12 [q][12] over t in [0, t_max].  Additive CCD with
 * zero thickness and gap fraction s in (0, 1): toi [q] receives a time at
 * which the pair is still separated by at least s times its initial gap and
 * before any contact, hit [q] = 1; or hit [q] = 0 and toi [q] = t_max when
 * the pair cannot meet before t_max.  max_iter caps the steps per pair
 * (reached: a hit at the time reached).  Host arrays; work runs on
 * dev->hip_stream and the call returns when it is done.  Errors: MS_E_ARG
 * (kinds, s, t_max, max_iter), MS_E_NONFINITE, MS_E_NOMEM, MS_E_DEVICE. */
ms_status ms_contact_toi(const ms_device* dev, int64_t n_pairs, const int32_t* kind, const double* x12,
                         const double* p12, double s, double t_max, int32_t max_iter, double* toi, int32_t* hit);

/* The self-contact constraint set (IPC's point-triangle and edge-edge
 * pairs closer than d_hat) on the GPU without a context.  x [n_verts][3];
 * the surface: vertices sverts [n_sverts], triangles tris [n_tris][3] and
 * edges edges [n_edges][2] (vertex ids).  Boxes inflated by d_hat / 2 are
 * entered into a grid of cell size `cell` (<= 0: the largest primitive
 * extent plus d_hat), pairs sharing a cell are deduplicated and kept when
 * their exact distance is below d_hat (a vertex is never paired with a
 * triangle containing it, nor an edge with one sharing a vertex).  *out
 * receives an opaque result that ms_pairs_get queries (first with null
 * arrays, then with pt [n_pt][2] = (vertex id, triangle index) and
 * ee [n_ee][2] = (edge index i, edge index j > i), both in ascending order)
 * and ms_pairs_free releases.  Host arrays; work runs on dev->hip_stream.
 * Errors: MS_E_ARG (indices, d_hat, a scene too large for the grid or
 * spanning 2^31 cells or more),
 * MS_E_NONFINITE, MS_E_NOMEM, MS_E_DEVICE. */
typedef struct ms_pairs ms_pairs;
ms_status ms_contact_pairs(const ms_device* dev, int64_t n_verts, const double* x, int64_t n_sverts,
                           const int32_t* sverts, int64_t n_tris, const int32_t* tris, int64_t n_edges,
                           const int32_t* edges, double dhat, double cell, ms_pairs** out);
ms_status ms_pairs_get(const ms_pairs* p, int64_t* n_pt, int32_t* pt, int64_t* n_ee, int32_t* ee);
void ms_pairs_free(ms_pairs* p);

/* Select how every later coarse matrix (two-level preconditioners, paper
 * mode's subspace level, ms_eval) is integrated (ms_coarse_integration).
 * Errors: MS_E_ARG, MS_E_ORDER (MS_COARSE_CUBATURE without a cubature). */
ms_status ms_set_coarse_integration(ms_ctx* c, int32_t mode);

/* Advance one timestep of size dt (s) with parameters p (NULL = defaults);
 * stats may be NULL.  Transactional: on any error x, v, the BDF2 history and
 * the warm start's coarse history are unchanged.
 * Errors: MS_E_ARG (dt not positive, parameters out of range, BDF2 with
 * paper mode or with the learned warm start, the smoothed two-level form
 * with the cubature coarse matrix), MS_E_ORDER (no state; a two-level
 * preconditioner or paper mode without a basis), MS_E_NOCONV,
 * MS_E_LINESEARCH (no decrease within max_backtracks halvings, or no
 * descent direction), MS_E_NONFINITE, MS_E_DEVICE. */
ms_status ms_step(ms_ctx* c, double dt, const ms_solver_params* p, ms_step_stats* stats);

/* Coarse coordinates of the current state: q = (U^T M U)^{-1} U^T M (x - x_rest),
 * [12 m] doubles (the handles of Eq. LBS).  Requires a basis. */
ms_status ms_get_coarse(ms_ctx* c, double* q);

/* ---- learned coarse warm start ------------------------------------------
 * A 3-layer MLP in -> width -> width -> out with SiLU activations, BF16
 * weights and FP32 accumulation, predicting the next coarse state from the
 * last two (in = 2 * 12 m, out = 12 m).  Weights are row-major [out][in]
 * FP32 on the host (rounded to BF16 on upload); mean/std standardise the
 * input, out_scale rescales the output; the prediction is a residual over
 * the constant-velocity extrapolation 2 q^t - q^{t-1}. */
typedef struct {
  int32_t in_dim, width, out_dim;
  const float *W0, *b0, *W1, *b1, *W2, *b2;
  const float *in_mean, *in_std, *out_scale;
} ms_mlp_desc;
ms_status ms_set_warmstart(ms_ctx* c, const ms_mlp_desc* d);
/* Install the network (NULL removes it).  Requires a basis; in_dim = 2 r,
 * out_dim = r, r = 12 m.  Weights are copied.  The prediction is used by
 * ms_step with warm_start = 1 once two coarse states are recorded (the
 * history restarts at ms_set_state), and only if it lowers the energy;
 * otherwise the step starts as without it.  Errors: MS_E_ORDER (no basis),
 * MS_E_ARG (shapes, non-positive std), MS_E_NONFINITE. */

/* The network on the GPU without a context (training and parity checks).
 * params: the six arrays W0 [w][in], b0 [w], W1 [w][w], b1 [w],
 * W2 [out][w], b2 [out] concatenated, FP32 host.  Products run on bf16
 * matrix cores with FP32 accumulation.  Work runs on dev->hip_stream.
 * ms_mlp_forward: Z [n][in] (already standardised) -> Y [n][out].
 * ms_mlp_train: Adam (beta 0.9 / 0.999, eps 1e-8, bias-corrected, FP32
 * master weights) on the mean squared error; step s uses the samples
 * order[s * batch .. (s+1) * batch) of X [n_samples][in], T [n_samples][out];
 * params are updated in place; losses [n_steps] (optional) receives each
 * step's loss before its update and first_grads (optional, same layout as
 * params) the gradient of the first step.  Errors: MS_E_ARG (shapes,
 * indices out of range), MS_E_NOMEM, MS_E_DEVICE. */
ms_status ms_mlp_forward(const ms_device* dev, int32_t in_dim, int32_t width, int32_t out_dim, const float* params,
                         int64_t n, const float* Z, float* Y);
ms_status ms_mlp_train(const ms_device* dev, int32_t in_dim, int32_t width, int32_t out_dim, float* params,
                       int64_t n_samples, const float* X, const float* T, int32_t n_steps, int32_t batch,
                       const int32_t* order, float lr, float* losses, float* first_grads);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward pass of ms_mlp_forward on DEVICE buffers the caller owns --
 * params (the concatenated FP32 weights of ms_mlp_forward), Z [n][in] and
 * Y [n][out] -- that calls no allocator of any kind.  The activations live
 * in one library-owned device array of MS_MLP_NOALLOC_SCRATCH_FLOATS floats
 * per GPU (held until the process ends), so 4 n width must not exceed it.
 * Asynchronous: the work is enqueued on dev->hip_stream and Y is ready when
 * the stream reaches it (no synchronisation, so the call can be captured).
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams or host threads) race.  Errors: MS_E_ARG (null
 * pointers, sizes, 4 n width above the limit), MS_E_DEVICE. */
#define MS_MLP_NOALLOC_SCRATCH_FLOATS (1 << 20)
ms_status ms_mlp_forward_noalloc(const ms_device* dev, int32_t in_dim, int32_t width, int32_t out_dim,
                                 const float* params, int64_t n, const float* Z, float* Y);

/* ---- kernel-level entry points (parity checks and measurements) ---------
 * ms_eval: at positions x [n][3] (host), with x~ = x^t + dt v^t from the
 * current state, return the energy parts e4 = {K, h^2 Psi, h^2 G, h^2 B},
 * the gradient grad [n][3] (Dirichlet DOFs NOT eliminated) and, if hess
 * is non-null, the PSD-projected Hessian as BSR3 values [nnzb][3][3] in the
 * pattern returned by ms_get_pattern.  prec selects the Hessian precision.
 * With self-contact, B includes its barrier and grad its forces; hess holds
 * the blocks of the mesh pattern only (couplings of vertices that share no
 * tet sit in the contact slots, outside it).  ms_energy_difference adds the
 * self-contact difference to dB. */
ms_status ms_get_pattern(const ms_ctx* c, int64_t* nnzb, int32_t* row_ptr, int32_t* col);
ms_status ms_eval(ms_ctx* c, const double* x, double dt, int32_t prec, double* e4, double* grad,
                  double* hess);

/* Energy difference E(x + alpha d) - E(x) of the incremental potential
 * (Eq. IP with the implicit Euler inertia term), with x~ from the current
 * state, evaluated term by term so that the large totals never cancel:
 * parts5 = {dK, h^2 dPsi, h^2 dG, h^2 dB, magnitude}, where magnitude is the
 * sum of the absolute values of the terms (the scale of the round-off in
 * the sum of the first four).  This is the quantity the line search tests
 * the Armijo condition on.  x, d [n][3] host.  Errors: MS_E_ORDER before
 * ms_set_state, MS_E_NONFINITE for non-finite x or d. */
ms_status ms_energy_difference(ms_ctx* c, const double* x, const double* d, double alpha, double dt,
                               double* parts5);

/* Apply the preconditioner built for the Hessian of the last ms_eval
 * (kind = ms_preconditioner) to r [n][3]; z [n][3].  Dirichlet DOFs of z
 * are zero. */
ms_status ms_apply_preconditioner(ms_ctx* c, int32_t kind, int32_t prec, const double* r, double* z);

/* Coarse operator U^T H U (12m x 12m, row-major) of the last ms_eval. */
ms_status ms_get_coarse_matrix(ms_ctx* c, double* A);

/* Measurement of kernel 0, the PCG product w = H u fused with the dots
 * (r.u, w.u, r.r) that every PCG iteration runs, in precision prec.
 * reps > 0: average duration in microseconds of `reps` back-to-back launches
 * on the context's stream, bracketed by HIP events, on the Hessian of the
 * last assembly (overwrites PCG scratch vectors).  reps = 0: average over
 * the launches recorded inside the PCG solves of ms_step calls made with
 * time_kernels = 1 (launches after convergence excluded), then the record
 * is cleared.  *bytes receives the kernel's algorithmic bytes per launch
 * (matrix values and column indices of the stored blocks, slice offsets,
 * u and r read, w written, Dirichlet mask; each counted once).
 * kernel 1..5 (reps > 0 only) replays the other kernels of a PCG iteration
 * on the current buffers: 1 the update (p, s, d, r, u), 2 the restriction
 * c = U^T r, 3 the coarse GEMV e = A^-1 c, 4 the prolongation u += U e,
 * 5 one whole iteration (bytes 0: not a single kernel).  These overwrite
 * the PCG vectors.  kernel 6 (reps > 0) replays the integration of the
 * coarse matrix U^T H U on the last assembled Hessian with the selected
 * ms_coarse_integration (bytes 0); it leaves the coarse factor to be
 * rebuilt by the next step.
 * Errors: MS_E_ORDER (nothing assembled / recorded yet, or no basis for
 * 2..4), MS_E_ARG. */
ms_status ms_time_kernel(ms_ctx* c, int32_t kernel, int32_t prec, int32_t reps, double* avg_us, double* bytes);

/* ---- standalone sliced-BSR3 matrix for SpMV measurements ----------------
 * A block-sparse matrix with 3x3 blocks given in BSR form (host row_ptr
 * [n+1], col [nnzb], vals [nnzb][3][3] doubles) is converted into the
 * library's device layout (slices of 16, 32 or 64 rows: MS_SLICE, else the
 * fastest on this pattern; component-major planes) in FP64
 * (dtype 0) or FP32 (dtype 1).  ms_mat_spmv computes y = A x for DEVICE
 * vectors x, y of 3n elements of that dtype on the matrix's stream. */
typedef struct ms_mat ms_mat;
ms_status ms_mat_create(const ms_device* dev, int64_t n, const int32_t* row_ptr, const int32_t* col,
                        const double* vals, int32_t dtype, ms_mat** out);
ms_status ms_mat_spmv(ms_mat* A, const void* x_dev, void* y_dev);
/* Algorithmic bytes of one product (values, indices, x, y counted once). */
double ms_mat_bytes(const ms_mat* A);
void ms_mat_destroy(ms_mat* A);

/* ---- batched scenes ------------------------------------------------------
 * Many independent scenes advanced as one block-diagonal system with
 * per-scene reductions, masks, line searches and convergence (the batched
 * workload of uneven scenes; each scene's result equals ms_step on its own
 * context).  Supported: plain implicit-Euler steps with block-Jacobi or
 * the additive two-level preconditioner (every scene with an installed
 * basis and the exact coarse matrix; each keeps its own coarse operator),
 * FP64 or mixed precision (one Hessian precision per step: no FP64
 * endgame), and the IPC half-space barrier when every scene has the same
 * half-space (no friction); each scene's line search starts from its own
 * CCD bound.
 *
 * ms_batch_create: join the contexts scenes[n_scenes] (states set, one
 * device, the same gravity, no context twice) into a batch *out; the union
 * of their meshes is built here once.  The batch refers to the contexts,
 * which must outlive it; their Dirichlet targets and states may change
 * between steps, their meshes not.  Errors: MS_E_ARG, MS_E_ORDER (a scene
 * without state), MS_E_NOMEM, MS_E_DEVICE.
 * ms_batch_advance: one timestep of every scene of the batch (per_scene
 * [n_scenes] may be NULL).  Errors: as ms_step, and MS_E_ORDER if a scene's
 * mesh changed since ms_batch_create.
 * ms_batch_step: the same step on a list of contexts in one call (the union
 * is cached on the first context and rebuilt when the list changes). */
typedef struct ms_batch ms_batch;
ms_status ms_batch_create(ms_ctx* const* scenes, int32_t n_scenes, ms_batch** out);
ms_status ms_batch_advance(ms_batch* b, double dt, const ms_solver_params* p, ms_step_stats* per_scene);
void ms_batch_destroy(ms_batch* b);
ms_status ms_batch_step(ms_ctx* const* scenes, int32_t n_scenes, double dt, const ms_solver_params* p,
                        ms_step_stats* per_scene);

const char* ms_last_error(const ms_ctx* c);
void ms_destroy(ms_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* MS_H */
