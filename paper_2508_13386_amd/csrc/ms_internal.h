// Internal state of an ms_ctx and declarations shared by the library's
// translation units.  Device layouts:
//   * positions / vectors: [n][3] doubles (or floats in the FP32 parts);
//   * Hessian: sliced BSR3 ("SBSR3"): rows are grouped in slices of S
//     consecutive vertices (S = 16, 32 or 64, chosen per mesh by timing);
//     slice s holds width_s block columns; block k of row (S s + r) stores its
//     9 components at
//       vals[9 * base_s + (9 k + c) * S + r],  base_s = S * sum_{s'<s} width_s',
//     and its column at col[base_s + S k + r] (-1 for padding).  One wave
//     serves one slice with 64 / S lanes per row, so a load of component c
//     touches 64 / S runs of S consecutive values.
//   * per-tet element blocks: 10 blocks (a <= b of the 4 local vertices) of
//     3x3, [T][10][9], written by the element kernel and gathered without
//     atomics into the slots above.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ms.h"

namespace ms {

// Start of the 9 values of the block in slot `slot` (component stride S).
__host__ __device__ inline int64_t vbase(int64_t slot, int S) { return 9 * slot - 8 * (slot & (S - 1)); }

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Sliced BSR3 pattern on the device plus host copies needed by queries.
struct Pattern {
  int S = 64;  // slice height
  int maxw = 0;  // largest slice width
  int64_t n = 0, nnzb = 0, nslots = 0, nslices = 0;
  int32_t* d_slice_base = nullptr;   // [nslices+1] block-slot base of each slice (multiple of 64)
  int32_t* d_col = nullptr;          // [nslots]
  int32_t* d_diag_slot = nullptr;    // [n] slot of the diagonal block of each row
  std::vector<int32_t> h_row_ptr, h_col;  // canonical BSR (sorted columns)
  std::vector<int64_t> h_slot_of_bsr;     // [nnzb] slot of every canonical block
  std::vector<int32_t> h_slice_base;
};

// Cubature of the elastic part of the coarse matrix (Sec. 3.8): the selected
// tets with their weights and the device lists of its two-stage product.
struct Cubature {
  std::vector<int32_t> tets;     // ascending
  std::vector<double> w;         // weights (volume units)
  bool present = false;
  bool built = false;            // device lists match the basis and Dirichlet set
  int64_t nz = 0;                // stage-1 rows
  int4* d_info = nullptr;        // [nz] {tet, local a, first, end} or {-1 - v, k_v, 0, 0}
  double* d_scale = nullptr;     // [nz] w / V of the row's tet
  int32_t* d_ent = nullptr;      // [L][2] (local b, k_b)
  double* d_Z = nullptr;         // [nz][36]
  int32_t npairs = 0;
  int32_t* d_pair_ij = nullptr;  // [npairs][2]
  int32_t* d_pair_ptr = nullptr; // [npairs+1]
  int32_t* d_pair_ent = nullptr; // [L2][2] (k_v, z)
};

// One block of the block-diagonal coarse GEMV of a batch: kGemvRows rows of
// one scene's coarse inverse.
struct GemvSeg {
  const void* A;  // the scene's inverse (float in mixed precision, else double)
  int ld, r;      // its leading dimension and coarse size
  int row0;       // first scene row of the block
  int h0;         // first union handle of the scene
  int scene;
  int pad[2];
};

struct CubatureParams {
  double tol;
  int32_t n_init, n_add, max_rounds;
  uint64_t seed;
  int32_t n_threads;
};

struct Basis {
  int32_t m = 0;
  int64_t nnz = 0;
  std::vector<double> origins;    // [m][3]
  std::vector<int64_t> vptr;      // [n+1]
  std::vector<int32_t> vhandle;   // [nnz]
  std::vector<double> vphi;       // [nnz]
  std::vector<int32_t> part;      // [T] or empty
  // device: per-vertex rows and per-handle columns (transpose) of U
  int32_t* d_vptr = nullptr;      // [n+1]
  int32_t* d_vh = nullptr;        // [nnz]
  double* d_vw = nullptr;         // [nnz][4] = phi * [1, x - o_i]
  float* d_vw32 = nullptr;
  int32_t* d_hptr = nullptr;      // [m+1]
  int32_t* d_hv = nullptr;        // [nnz] vertex of each (handle, vertex) pair
  int32_t* d_hk = nullptr;        // [nnz] index into the per-vertex arrays
  // restriction: entries in handle order with their weights, split into
  // chunks of at most 1024 entries; chunk q is described by
  // chunk_info[q] = {handle, first entry, end entry, 0}; handle i owns the
  // hinfo[i].y chunks starting at hinfo[i].x
  double* d_hw = nullptr;         // [nnz][4] W of entry e (handle order)
  int32_t nrchunks = 0;
  int4* d_chunk_info = nullptr;   // [nrchunks]
  int2* d_hinfo = nullptr;        // [m]
  double* d_rpart = nullptr;      // [nrchunks][12] chunk partials
  // Galerkin lists.  Stage 1 (Z = H U): one entry per (v, j in h'(v)) with
  // its (Hessian slot, k_w) contributions; stage 2 (U^T Z): one entry per
  // coarse pair (i <= j) with its (k_v, z) contributions.
  int64_t nz = 0, z_L = 0;
  int32_t* d_zptr = nullptr;      // [nz+1]
  int32_t* d_zent = nullptr;      // [z_L][2]
  uint8_t* d_zmask = nullptr;     // [nz] 1 on Dirichlet rows
  double* d_Z = nullptr;          // [nz][36]
  int32_t npairs = 0;
  int32_t* d_pair_ij = nullptr;   // [npairs][2]
  int32_t* d_pair_ptr = nullptr;  // [npairs+1]
  int32_t* d_pair_ent = nullptr;  // [pair_L][2]
  int64_t pair_L = 0;
  double* d_Minv = nullptr;       // (U^T M U)^-1, [r][r]
};

}  // namespace ms

struct Mlp;

namespace ms {
// IPC self-contact between the mesh's own surface primitives (Sec. 4): the
// surface, the contact slots reserved in the Hessian pattern, and the lists
// of the current constraint set (rebuilt at every assembly).
struct SelfContact {
  bool on = false;
  double dhat = 0.0, kappa = 0.0;
  double cell = 0.0;  // broad-phase grid cell of the static constraint set
  int spare = 0;      // contact slots reserved per surface row
  std::vector<int32_t> h_tris, h_edges, h_verts;  // surface triangles [F][3], edges [E][2], vertices
  int32_t *d_tris = nullptr, *d_edges = nullptr, *d_verts = nullptr;
  std::vector<int32_t> h_spare0;  // [n] first contact slot (block column index) of each row, -1 none
  std::vector<int32_t> h_col;     // host copy of every slot's column, contact slots included
  double* d_y = nullptr;          // [3n] trial positions
  // lists of the last assembly: pair quads, gradient and Hessian gathers
  int64_t np = 0, ng = 0, nh = 0;
  int32_t* d_quad = nullptr;  // [np][5] kind (0 point-triangle, 1 edge-edge), four vertex ids
  double* d_pdat = nullptr;   // [np][24] energy, gradient [12], GN weight, coefficients [4], normal [3]
  int32_t* d_glist = nullptr; // ng vertices, ng + 1 offsets, entries [2] (pair, local)
  int32_t* d_hlist = nullptr; // nh slots, nh + 1 offsets, entries [3] (pair, local a, local b)
  int32_t* d_aux = nullptr;   // quads of energy evaluations and CCD candidates
  double* d_aux_out = nullptr;
  int64_t cap_quad = 0, cap_pdat = 0, cap_glist = 0, cap_hlist = 0, cap_aux = 0, cap_aux_out = 0;
};
}  // namespace ms

struct ms_ctx {
  ms_device dev{};
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;  // every live device allocation of this context
  std::string err;
  int stage = 0;  // 1 mesh, 2 material, 3 state
  // sizes
  int64_t n = 0, T = 0;
  // host mesh
  std::vector<double> h_rest;
  std::vector<int32_t> h_tets;
  std::vector<double> h_vol, h_mu, h_lam, h_mass, h_Dminv;
  std::vector<double> h_nu, h_rho;  // material as uploaded (batches rebuild from it)
  std::vector<double> h_E;
  double bbox_diag = 1.0;
  // device mesh
  double* d_rest = nullptr;
  int32_t* d_tets = nullptr;
  double* d_Dminv = nullptr;  // [T][9]
  double* d_vol = nullptr;
  double* d_mu = nullptr;
  double* d_lam = nullptr;
  double* d_mass = nullptr;
  int32_t* d_vt_ptr = nullptr;   // [n+1] vertex -> incident (tet, local) codes
  int32_t* d_vt_code = nullptr;  // [4T]  t*4 + a
  ms::Pattern pat;
  int32_t* d_gptr = nullptr;     // [nslots+1] gather ranges per slot
  int32_t* d_gcode = nullptr;    // [16T] (t*10 + pair)*2 + transpose
  // physics
  double gravity[3] = {0, 0, 0};
  bool has_hs = false;
  double hs_n[3] = {0, 0, 1}, hs_off = 0, hs_dhat = 1e-3, hs_kappa = 0;
  double hs_mu = 0.0, hs_epsv = 1e-3;  // lagged friction against the half-space
  double step_h = 0.0;                 // timestep of the current step / evaluation
  int proj_mode = 0;                   // projected element Hessians: 0 clamp, 1 absolute value
  int smoother = 0;                    // PCG block smoother of this step: 0 3x3 vertex blocks, 1 aggregates
  int cg_graph_smoother = 0;           // smoother the captured PCG graphs were recorded with
  // vertex aggregates of the aggregate block-Jacobi smoother (built from the
  // rest positions and the mesh pattern; stale once the pattern is rebuilt)
  struct Aggregates {
    bool built = false;
    int nagg = 0;
    int32_t* d_vert = nullptr;  // [nagg][kAggV] vertex ids, -1 padding
    int32_t* d_slot = nullptr;  // [nagg][kAggV][kAggV] slot of block (i, j), -1 none
    double* d_inv64 = nullptr;  // [nagg][kAggN][kAggN] inverse of the aggregate's diagonal block
    float* d_inv32 = nullptr;   // FP32 copy (mixed precision)
  } agg;
  ms::SelfContact sc;
  // basis build: local solves with at least this many unknowns run on the
  // GPU (0: host only); solves done there in the last build
  int basis_gpu_min = 0;
  int basis_gpu_solves = 0;
  double basis_seconds = 0.0;  // host wall time of the last ms_build_basis
  // Dirichlet
  std::vector<int32_t> h_dbc;
  std::vector<double> h_dbc_tgt;
  uint8_t* d_pinned = nullptr;
  int32_t* d_dbc = nullptr;
  double* d_dbc_tgt = nullptr;
  int64_t dbc_cap = 0;
  // state
  double* d_x = nullptr;
  double* d_v = nullptr;
  double* d_xt = nullptr;
  double* d_xtilde = nullptr;
  // BDF2 history: x^{t-1}, v^{t-1} of the last plain step (valid if has_prev)
  double* d_xprev = nullptr;
  double* d_vprev = nullptr;
  bool has_prev = false;
  double* d_xtrial = nullptr;
  // assembly workspace
  double* d_He = nullptr;     // [T][10][9] FP64
  float* d_He32 = nullptr;    // [T][10][9] FP32
  double* d_ge = nullptr;     // [T][12]
  double* d_g = nullptr;      // [n][3]
  double* d_vals = nullptr;   // sliced values FP64 [9*nslots]
  float* d_vals32 = nullptr;  // sliced values FP32
  double* d_Dinv = nullptr;   // [n][9] inverse diagonal blocks
  float* d_Dinv32 = nullptr;
  // PCG workspace
  double *d_d = nullptr, *d_r = nullptr, *d_u = nullptr, *d_w = nullptr, *d_p = nullptr, *d_s = nullptr;
  double* d_scal = nullptr;   // device scalars of the solvers
  double* h_scal = nullptr;   // pinned host mirror
  double* d_part = nullptr;   // reduction partials
  double* d_cgst = nullptr;   // PCG recurrence state, two buffers
  unsigned* d_counter = nullptr;
  int nblk_vert = 0;          // blocks of the per-vertex kernels
  // graphs of fixed-size PCG chunks (per precision x preconditioner)
  hipGraphExec_t cg_graph[2][4] = {{nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr, nullptr}};
  // mixed-precision steps: the PCG iterations that run with the FP64
  // Hessian also apply the FP32 coarse inverse (the FP64 graphs are captured
  // under the current value; set_coarse_f32 drops them when it changes)
  bool coarse_f32 = false;
  int cg_chunk = 16;
  bool use_graphs = true;
  bool own_stream = false;
  int verbose = 0;
  // basis / two-level preconditioner
  ms::Basis basis;
  bool has_basis = false;
  int32_t r = 0;              // 12 m
  double* d_c = nullptr;      // coarse rhs [r]
  double* d_e = nullptr;      // coarse solution [r]
  double* d_Ac = nullptr;     // coarse matrix [r][r] (row-major), then its Cholesky factor
  double* d_Ainv = nullptr;   // explicit inverse of the coarse matrix [r][r]
  float* d_Ainv32 = nullptr;  // its symmetrised FP32 copy (mixed precision)
  int32_t rp = 0;             // r padded to the factorisation tile
  double* d_Lc = nullptr;     // Cholesky factor workspace [rp][rp]
  double* d_Y = nullptr;      // inverse factor workspace [rp][rp]
  double* d_Ldiag = nullptr;  // factored diagonal tiles
  double* d_Linvd = nullptr;  // inverses of the factored diagonal tiles
  double* d_diag0 = nullptr;  // regularised diagonal [r]
  int* d_nreg = nullptr;      // regularised pivots
  float* d_Ac32 = nullptr;    // FP32 Galerkin accumulation
  double* d_cpart = nullptr;  // coarse restriction partials
  int coarse_valid = 0;
  // coarse matrix: exact Galerkin product or the cubature of its elastic part
  ms::Cubature cub;
  int coarse_mode = MS_COARSE_EXACT;
  const double* asm_x = nullptr;  // positions and h^2 of the last assembly
  double asm_h2 = 0.0;
  // learned warm start
  Mlp* mlp = nullptr;
  std::vector<double> q_prev, q_cur;  // last two coarse states
  int q_hist = 0;
  // last eval
  int eval_prec = 0;
  bool eval_valid = false;
  bool assembled[2] = {false, false};  // a Hessian of that precision is in place
  struct BatchPlan* batch = nullptr;  // cached union of the last ms_batch_step's scenes (owned)
  // paper mode (Alg. 1 and 2)
  void* d_lag = nullptr;       // lagged elastic + inertia part of H, [slots][9] in the mode's value type
  void* d_hlag = nullptr;      // H_lag = lag + barrier curvature at the current x
  void* d_Dinv_lag = nullptr;  // 3x3 block-Jacobi inverses of H_lag
  int lag_prec = -1;           // value type the lag buffers were allocated for
  double* d_ds = nullptr;      // subspace direction d_s [n][3]
  double* d_gsave = nullptr;   // gradient saved across the refinement solve
  double* d_paper = nullptr;   // subspace-level workspace (coarse vectors, A C, block inverses, PCG state)
  int paper_r = -1;            // coarse size d_paper was laid out for
  std::vector<double> h_delta; // handle-origin offsets from the affine origin [m][3]
  double oa[3] = {0, 0, 0};    // origin of the affine basis (rest centre of mass)
  int refine_auto = 20;        // refinement iterations from the partition hop diameter
  // live timing of the PCG product (time_kernels)
  bool timing = false;
  std::vector<hipEvent_t> tev;      // 2 per iteration of a chunk
  double timed_ms[2] = {0.0, 0.0};  // per precision: accumulated duration
  int64_t timed_n[2] = {0, 0};
};

struct ms_mat {
  ms_ctx ctx;  // reuses the allocator / stream plumbing of a context
  int dtype = 0;
  double bytes = 0.0;
};

namespace ms {

// error helpers ------------------------------------------------------------
ms_status fail(ms_ctx* c, ms_status s, const std::string& msg);
ms_status hip_fail(ms_ctx* c, hipError_t e, const char* what);
#define MS_HIP(call)                                    \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ms::hip_fail(c, e_, #call); \
  } while (0)

void* dalloc(ms_ctx* c, size_t bytes);
void dfree(ms_ctx* c, void* p);
template <class T>
ms_status alloc_n(ms_ctx* c, T** p, size_t n) {
  if (*p) dfree(c, *p);
  *p = static_cast<T*>(dalloc(c, n * sizeof(T) + 256));
  if (!*p) return fail(c, MS_E_NOMEM, "device allocation failed");
  return MS_OK;
}
template <class T>
ms_status upload(ms_ctx* c, T** p, const T* h, size_t n) {
  ms_status s = alloc_n(c, p, n);
  if (s) return s;
  if (n) {
    hipError_t e = hipMemcpyAsync(*p, h, n * sizeof(T), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync H2D");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  }
  return MS_OK;
}

// host precompute (mesh.cpp, basis.cpp) -------------------------------------
ms_status mesh_geometry(ms_ctx* c);
ms_status build_mesh(ms_ctx* c);
ms_status build_pattern(ms_ctx* c);
void slice_layout(int64_t n, const int32_t* row_ptr, int S, std::vector<int32_t>& slice_base, int& maxw);
double time_spmv_layout(ms_ctx* c, int S, const int32_t* d_slice_base, const int32_t* d_col, int64_t nslices,
                        int64_t nslots, int reps);
ms_status build_basis_host(ms_ctx* c, const ms_basis_params& P, Basis& B);
ms_status install_basis(ms_ctx* c, Basis&& B);
ms_status install_transfer(ms_ctx* c, const Basis& B);
void launch_coarse_gemv_seg(ms_ctx* u, int prec, const GemvSeg* seg, int nblocks_seg, int rmax, const double* sscal,
                            int sstride);
constexpr int kGemvRowsPerBlock = 16;  // rows per block of the coarse GEMV kernels
ms_status coarse_coordinates(ms_ctx* c, const double* x_dev, double* q_host, double* q_dev);

// kernel launchers (kernels_*.hip) -------------------------------------------
enum Scal {  // indices into ctx->d_scal
  S_GAMMA = 0, S_DELTA, S_RHO, S_ALPHA, S_BETA, S_GAMMA_OLD, S_ALPHA_OLD, S_ITER, S_DONE, S_TOL2,
  S_RHO0, S_MAXIT, S_E0, S_E1, S_E2, S_E3, S_CCD, S_DOT0, S_DOT1, S_DOT2, S_G0SQ, S_GPREV, S_ETAPREV, S_ETA,
  S_DE0, S_DE1, S_DE2, S_DE3, S_DE4,
  S_COUNT = 32
};

void launch_predict(ms_ctx* c, double dt);
void launch_apply_dbc(ms_ctx* c, int64_t nd);
void launch_element(ms_ctx* c, const double* x, double h2, int prec, bool hess, bool project,
                    const int32_t* tscene = nullptr, const uint8_t* sproj = nullptr);
void launch_gather_grad(ms_ctx* c, const double* x, double h2, double* g);
void launch_gather_hess(ms_ctx* c, const double* x, double h2, int prec);
void launch_block_jacobi(ms_ctx* c, int prec);
void launch_energy(ms_ctx* c, const double* x, const double* d, double alpha, double h2);
void launch_energy_delta(ms_ctx* c, const double* x, const double* d, double alpha, double h2);
void launch_ccd(ms_ctx* c, const double* x, const double* d);
void launch_dots(ms_ctx* c, const double* a, const double* b, const double* a2, const double* b2,
                 const double* a3, const double* b3);
void launch_axpy(ms_ctx* c, double* y, const double* x, double alpha, int64_t len);
void launch_velocity(ms_ctx* c, double inv_h);
void launch_predict_bdf2(ms_ctx* c, double dt);
void launch_velocity_hist(ms_ctx* c, double dt, bool bdf2);
void launch_cg_init(ms_ctx* c, int prec, double eta_max, double eta_min, bool first, int max_it, int forcing);
void launch_coarse_correction(ms_ctx* c, int prec, bool from_w);
void launch_precond_apply(ms_ctx* c, int prec, int pc);
void launch_coarse_start(ms_ctx* c, int prec);
void launch_spmv_resid(ms_ctx* c, int prec, bool from_d);
void launch_bj(ms_ctx* c, int prec);
void launch_prolong_set_d(ms_ctx* c);
inline bool two_level(int pc) {
  return pc == MS_PC_TWO_LEVEL || pc == MS_PC_TWO_LEVEL_ADDITIVE || pc == MS_PC_TWO_LEVEL_VCYCLE;
}
constexpr int kUpdBlock = 256;  // vertices per PCG update block
constexpr int kAggV = 8;                // vertices per aggregate (at most)
constexpr int kAggN = 3 * kAggV;        // DOFs per aggregate
ms_status build_aggregates(ms_ctx* c);
void launch_agg_invert(ms_ctx* c, int prec);
void launch_agg_apply(ms_ctx* c, int prec);
void launch_cg_update_agg(ms_ctx* c, int prec, int parity);
void launch_coarse_gemv(ms_ctx* c, int prec, const double* scal);
void launch_prolong_add(ms_ctx* c, double* target, const double* scal);
void launch_diag_barrier(ms_ctx* c, int prec, void* vals, const double* x, double h2, double sign);
void set_coarse_f32(ms_ctx* c, bool on);
void launch_block_jacobi_l1(ms_ctx* c, int prec);
void launch_bj_add(ms_ctx* c, int prec);
void launch_restrict(ms_ctx* c, const double* v, const double* weight, const double* scal);
void launch_cg_update(ms_ctx* c, int prec, int parity);
void destroy_batch(ms_ctx* c);
void destroy_mlp(ms_ctx* c);
ms_status time_loop_kernel(ms_ctx* c, int kernel, int prec, int reps, double* avg_us, double* bytes);
void launch_cg_iteration(ms_ctx* c, int prec, int pc, int parity, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_precond(ms_ctx* c, int pc, int prec, const double* r, double* z);
void launch_spmv(ms_ctx* c, int prec, const double* x, double* y);
ms_status launch_galerkin(ms_ctx* c, int prec, const double* x, double h2);
ms_status time_coarse_matrix(ms_ctx* c, int prec, int reps, double* avg_us, double* bytes);
ms_status fit_cubature_host(int64_t n, const double* rest, int64_t T, const int32_t* tets, const int32_t* part,
                            const int64_t* vptr, const int32_t* vhandle, const double* vphi,
                            const CubatureParams& P, std::vector<int32_t>& sel, std::vector<double>& wts,
                            double* max_rel);
ms_status build_cubature_lists(ms_ctx* c);
ms_status coarse_factor(ms_ctx* c);
int coarse_pad(int r);
void launch_extract_bsr(ms_ctx* c, const int64_t* slot_of_bsr_dev, int64_t nnzb, double* out, int prec);
void launch_fill(ms_ctx* c, double* p, double v, int64_t len);

// solver (api.hip, solver.hip)
ms_status sync(ms_ctx* c);
ms_status read_scal(ms_ctx* c);
ms_status pcg_solve(ms_ctx* c, int prec, int pc, double eta_max, double eta_min, bool first, int max_it, int* iters,
                    int* code, int forcing);
ms_status assemble(ms_ctx* c, const double* x, double h2, int prec, bool project, bool need_pc, int pc,
                   bool refresh_coarse);
ms_status energy(ms_ctx* c, const double* x, const double* d, double alpha, double h2, double parts[4]);
ms_status energy_delta(ms_ctx* c, const double* x, const double* d, double alpha, double h2, double* dE,
                       double* err);
ms_status plain_step(ms_ctx* c, double dt, const ms_solver_params& P, ms_step_stats* st);
ms_status paper_step(ms_ctx* c, double dt, const ms_solver_params& P, ms_step_stats* st);
void release_all(ms_ctx* c);
ms_status time_cg_spmv(ms_ctx* c, int prec, int reps, double* avg_us, double* bytes);
double cg_spmv_bytes(const ms_ctx* c, int prec);
ms_status line_search(ms_ctx* c, double h2, double gd, int max_bt, double* alpha_out, int* nbt);
ms_status warm_start(ms_ctx* c, double dt, bool inertial, int32_t* used);
ms_status inertial_start(ms_ctx* c, double h2);
ms_status try_move(ms_ctx* c, double h2);
void launch_predictor_dir(ms_ctx* c);
ms_status record_coarse(ms_ctx* c);
ms_status mat_build(struct ::ms_mat* A, int64_t n, const int32_t* row_ptr, const int32_t* col, const double* vals);

// dense SPD solve on the GPU (dense_chol.hip): A given as full symmetric
// CSR (n rows), rhs [n] host, overwritten by the solution; *ok false when a
// pivot was not positive (rhs then undefined)
ms_status dense_spd_solve(ms_ctx* c, int n, const int* ptr, const int* idx, const double* val, double* rhs,
                          bool* ok);

// multi-source geodesic Voronoi on the device (geodesic.hip): the basis
// build's edge graph (CSR with costs) and its sweep buffers
struct DevGraph {
  static constexpr int kSweepChunk = 8;  // sweeps between host looks at the change flags
  int n = 0;
  int *ptr = nullptr, *idx = nullptr;
  double* len = nullptr;
  double* d[2] = {nullptr, nullptr};
  int* l[2] = {nullptr, nullptr};
  int *flags = nullptr, *seeds = nullptr;
  ms_status upload(ms_ctx* c, const std::vector<int>& ptr, const std::vector<int>& idx,
                   const std::vector<double>& cost);
  // label [n] (index into seeds, -1 unreached) and distance of the nearest seed
  ms_status voronoi(ms_ctx* c, const std::vector<int>& seeds, std::vector<int>& label, std::vector<double>& dist);
  void release(ms_ctx* c);
};

// self-contact (selfcontact.hip)
ms_status sc_setup(ms_ctx* c);
ms_status sc_assemble(ms_ctx* c, const double* x, double h2, int prec);
ms_status sc_energy(ms_ctx* c, const double* x, double h2, double* e);
ms_status sc_energy_delta(ms_ctx* c, const double* x, const double* d, double alpha, double h2, double* dE,
                          double* err);
ms_status sc_ccd(ms_ctx* c, const double* x, const double* d, double* t);
void mat_spmv(struct ::ms_mat* A, const void* x, void* y);

}  // namespace ms
