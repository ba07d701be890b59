// Batched timesteps of many independent scenes in one set of launches.
//
// The scenes' meshes are joined into one disjoint union (a hidden context,
// built once per list of scenes and cached), with every scene's vertex
// range starting at a multiple of 256 (isolated, pinned, massless padding
// vertices fill the gaps).  Then every 32-row slice, every 4-slice product
// block and every 256-vertex update block belongs to exactly one scene, and
// a scene's blocks cover its vertices exactly as in its own context.  All
// kernels run once per stage over the union; what is per scene is
// segmented:
//   * PCG: each scene has its own recurrence state, tolerance, iteration
//     count and done flag; the product kernel skips blocks of finished
//     scenes, the update kernel reduces only its scene's dot partials, in
//     the same order as the single-scene reduction;
//   * Newton: per-scene line-search step (one energy-difference launch per
//     backtracking round evaluates every scene at its own alpha),
//     convergence test and exact-Hessian endgame flag (the element kernel
//     takes its projection choice from the tet's scene).
// With the reductions laid out this way each scene follows the arithmetic
// of its own unbatched ms_step; finished scenes idle while the others
// continue.  Supported: plain mode, block-Jacobi PCG, FP64 or mixed
// precision, no half-space contact.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cg_device.h"
#include "energy_device.h"
#include "ms_internal.h"
#include "reduce.h"

struct BatchPlan {
  std::vector<ms_ctx*> scenes;
  std::vector<int64_t> n_s, T_s;  // sizes the plan was built for
  std::vector<int64_t> v0, t0;    // vertex / tet offsets in the union
  std::vector<int64_t> npad;      // padded vertex count of each scene
  ms_ctx* u = nullptr;
  int ns = 0;
  int64_t nub = 0, nbs = 0, ebx = 0;  // update blocks, product blocks, energy blocks per scene
  int32_t* d_tscene = nullptr;    // [T] scene of each tet
  int32_t* d_pbscene = nullptr;   // [nbs] scene of each product block
  int32_t* d_ubscene = nullptr;   // [nub] scene of each update block
  int4* d_sinfo = nullptr;        // [ns] {first product block, count, first update block, count}
  int4* d_einfo = nullptr;        // [ns] {first tet, tets, first vertex, vertices}
  double* d_sscal = nullptr;      // [ns][S_COUNT]
  double* d_sst = nullptr;        // [2][ns][ST_N]
  double* d_salpha = nullptr;     // [ns]
  uint8_t* d_sproj = nullptr;     // [ns]
  uint8_t* d_sactive = nullptr;   // [ns]
  uint8_t* d_sfirst = nullptr;    // [ns]
  double* d_spart = nullptr;      // partials of the segmented reductions
  double* d_sout = nullptr;       // [ns][8] their results
  int2* d_drange = nullptr;       // [ns] dot-partial range of each scene (blocks of 256 entries of 3n)
  int2* d_erange = nullptr;       // [ns] energy-partial range of each scene
  hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [precision][two-level]
  std::vector<double> h_sscal;
  // two-level (additive) preconditioner: the union carries the transfer
  // operators of the scenes' bases; each scene keeps its coarse matrix
  bool tl_ready = false;
  std::vector<int32_t> h0;        // first union handle of each scene
  std::vector<int64_t> slot0;     // first union slot of each scene's slices
  ms::GemvSeg* d_seg[2] = {nullptr, nullptr};  // GEMV blocks reading FP64 / FP32 inverses
  int nseg = 0, rmax = 0;
  std::vector<double> moved;      // per scene: movement since the last coarse rebuild
  std::vector<const void*> tl_key;  // per scene: inverses and sizes the tables were built for
};

namespace ms {

namespace {

constexpr int kStride = S_COUNT;  // doubles of per-scene scalars

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// --- PCG -------------------------------------------------------------------

template <typename VT>
__global__ void __launch_bounds__(256) k_bcg_init(int64_t n, const double* __restrict__ g,
                                                  const uint8_t* __restrict__ pinned, double* __restrict__ p,
                                                  double* __restrict__ s, double* __restrict__ d,
                                                  double* __restrict__ r, double* __restrict__ u,
                                                  const VT* __restrict__ Dinv, double* __restrict__ part) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double rho[1] = {0.0};
  if (v < n) {
    const bool pin = pinned[v];
    double rr[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int64_t k = 3 * v + i;
      const double gi = pin ? 0.0 : -g[k];
      rr[i] = gi;
      r[k] = gi;
      p[k] = 0.0;
      s[k] = 0.0;
      d[k] = 0.0;
      rho[0] += gi * gi;
    }
    double uu[3];
    bj_apply<VT>(Dinv, v, rr, uu);
#pragma unroll
    for (int i = 0; i < 3; ++i) u[3 * v + i] = uu[i];
  }
  block_sum<1>(rho);
  if (threadIdx.x == 0) part[blockIdx.x] = rho[0];
}

// One block per scene: the initial residual, tolerance and flags (the
// forcing rules of the single-scene PCG).  Inactive scenes get done = 5.
__global__ void __launch_bounds__(256) k_bcg_init_finish(const int4* __restrict__ sinfo,
                                                         const double* __restrict__ part,
                                                         const uint8_t* __restrict__ active,
                                                         const uint8_t* __restrict__ first, double eta_max,
                                                         double eta_min, int forcing, double maxit,
                                                         double* __restrict__ sst, double* __restrict__ sscal) {
  const int sc = blockIdx.x;
  const int4 in = sinfo[sc];
  double acc[1] = {0.0};
  for (int b = threadIdx.x; b < in.w; b += blockDim.x) acc[0] += part[in.z + b];
  block_sum<1>(acc);
  if (threadIdx.x != 0) return;
  double* scal = sscal + kStride * sc;
  double* st0 = sst + ST_N * sc;
  const double rho0 = acc[0];
  const bool fst = first[sc] != 0;
  scal[S_RHO0] = rho0;
  scal[S_RHO] = rho0;
  if (fst) scal[S_G0SQ] = rho0;
  double eta;
  if (forcing == 1) {
    if (fst || !(scal[S_GPREV] > 0.0)) {
      eta = eta_max;
    } else {
      eta = 0.9 * rho0 / scal[S_GPREV];
      const double safe = 0.9 * scal[S_ETAPREV] * scal[S_ETAPREV];
      if (safe > 0.1) eta = fmax(eta, safe);
    }
  } else {
    eta = scal[S_G0SQ] > 0.0 ? sqrt(sqrt(rho0 / scal[S_G0SQ])) : 1.0;
  }
  eta = fmin(eta_max, fmax(eta_min, eta));
  if (active[sc]) {
    scal[S_GPREV] = rho0;
    scal[S_ETAPREV] = eta;
  }
  scal[S_ETA] = eta;
  scal[S_TOL2] = eta * eta * rho0;
  scal[S_ITER] = 0.0;
  scal[S_MAXIT] = maxit;
  st0[ST_GAMMA] = 0.0;
  st0[ST_ALPHA] = 1.0;
  st0[ST_ITER] = 0.0;
  scal[S_DONE] = !active[sc] ? 5.0 : (rho0 > 0.0 ? 0.0 : 1.0);
}

template <typename VT, int S>
__global__ void __launch_bounds__(256) k_bcg_spmv(int64_t n, int64_t nslices, const int32_t* __restrict__ slice_base,
                                                  const int32_t* __restrict__ scol, const VT* __restrict__ vals,
                                                  const double* __restrict__ u, double* __restrict__ w,
                                                  const double* __restrict__ r, const uint8_t* __restrict__ pinned,
                                                  const int32_t* __restrict__ pbscene,
                                                  const double* __restrict__ sscal, double* __restrict__ part) {
  const double done = sscal[kStride * pbscene[blockIdx.x] + S_DONE];
  const int64_t s = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t row = s * S + lane % S;
  const bool has = s < nslices;
  const int base = has ? slice_base[s] : 0;
  const int width = has ? (slice_base[s + 1] - base) / S : 0;
  if (done != 0.0) return;  // the same for every block of the scene
  double dots[3] = {0.0, 0.0, 0.0};
  if (has) {
    double acc[3];
    row_product_range<VT, double, S>(base, width, lane, scol, vals, u, acc);
    if (lane < S && row < n) {
      const bool pin = pinned[row];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double wi = pin ? 0.0 : acc[i];
        w[3 * row + i] = wi;
        const double ui = u[3 * row + i], ri = r[3 * row + i];
        dots[0] += ri * ui;
        dots[1] += wi * ui;
        dots[2] += ri * ri;
      }
    }
  }
  block_sum<3>(dots);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < 3; ++i) part[3 * blockIdx.x + i] = dots[i];
}

template <typename VT>
__global__ void __launch_bounds__(256) k_bcg_update(int64_t n, const int32_t* __restrict__ ubscene,
                                                    const int4* __restrict__ sinfo, const double* __restrict__ part,
                                                    const double* __restrict__ sst_in, double* __restrict__ sst_out,
                                                    double* __restrict__ p, double* __restrict__ s,
                                                    double* __restrict__ d, double* __restrict__ r,
                                                    double* __restrict__ u, const double* __restrict__ w,
                                                    const VT* __restrict__ Dinv, double* __restrict__ sscal) {
  const int sc = ubscene[blockIdx.x];
  double* scal = sscal + kStride * sc;
  const double done = scal[S_DONE];
  const int4 in = sinfo[sc];
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool own = v < n;
  double uo[3], po[3], wo[3], so[3], ro[3], dd[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int64_t k = own ? 3 * v + i : 0;
    uo[i] = u[k];
    po[i] = p[k];
    wo[i] = w[k];
    so[i] = s[k];
    ro[i] = r[k];
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) dd[q] = double(Dinv[own ? 9 * v + q : q]);
  if (done != 0.0) return;  // the same for every block of the scene
  double dots[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < in.y; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < 3; ++i) dots[i] += part[3 * (in.x + b) + i];
  block_sum<3>(dots);
  double alpha, beta;
  const double* st_in = sst_in + ST_N * sc;
  double* st_out = sst_out + ST_N * sc;
  const int code = cg_scalars(st_in, scal, dots[0], dots[1], dots[2], alpha, beta);
  if (int(blockIdx.x) == in.z && threadIdx.x == 0) {
    scal[S_RHO] = dots[2];
    if (code != 0) {
      scal[S_DONE] = double(code);
      scal[S_ITER] = st_in[ST_ITER];
    } else {
      st_out[ST_GAMMA] = dots[0];
      st_out[ST_ALPHA] = alpha;
      st_out[ST_ITER] = st_in[ST_ITER] + 1.0;
      scal[S_ITER] = st_in[ST_ITER] + 1.0;
    }
  }
  if (code != 0 || !own) return;
  double rr[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int64_t k = 3 * v + i;
    const double pi = uo[i] + beta * po[i];
    const double si = wo[i] + beta * so[i];
    p[k] = pi;
    s[k] = si;
    d[k] += alpha * pi;
    rr[i] = ro[i] - alpha * si;
    r[k] = rr[i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) u[3 * v + i] = dd[3 * i] * rr[0] + dd[3 * i + 1] * rr[1] + dd[3 * i + 2] * rr[2];
}

// --- Newton-level segmented reductions -------------------------------------

// Per-block partials of (a0.b0, a1.b1, |a2 - am2|^2) over blocks of 256
// vector entries (the blocks of the single-scene dot kernel).
__global__ void __launch_bounds__(256) k_bdots(int64_t len, const double* __restrict__ a0,
                                               const double* __restrict__ b0, const double* __restrict__ a1,
                                               const double* __restrict__ b1, const double* __restrict__ a2,
                                               const double* __restrict__ am2, double* __restrict__ part) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < len) {
    if (a0) v[0] = a0[i] * b0[i];
    if (a1) v[1] = a1[i] * b1[i];
    if (a2) {
      const double z = a2[i] - (am2 ? am2[i] : 0.0);
      v[2] = z * z;
    }
  }
  block_sum<3>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k) part[3 * blockIdx.x + k] = v[k];
}

// One block per scene: out[8 s + k] = sum of the scene's NV-value partials
// (first partial, count) in the order of the single-scene reduction.
template <int NV>
__global__ void __launch_bounds__(256) k_seg_finish(const int2* __restrict__ range, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  const int sc = blockIdx.x;
  const int2 rg = range[sc];
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < rg.y; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] += part[NV * (rg.x + b) + k];
  block_sum<NV>(acc);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) out[8 * sc + k] = acc[k];
}

// Energy difference at each scene's own step alpha_s; grid (blocks per
// scene, scenes): thread j of a scene takes its tet j and its vertex j, as
// thread j of the single-scene kernel does.
__global__ void __launch_bounds__(256) k_benergy_delta(const int4* __restrict__ einfo,
                                                       const int32_t* __restrict__ tets,
                                                       const double* __restrict__ Dminv,
                                                       const double* __restrict__ vol, const double* __restrict__ mu_,
                                                       const double* __restrict__ lam_,
                                                       const double* __restrict__ mass, const double* __restrict__ x,
                                                       const double* __restrict__ d,
                                                       const double* __restrict__ salpha,
                                                       const double* __restrict__ xtilde, double h2, double gx,
                                                       double gy, double gz, HalfSpace hs, double* __restrict__ part) {
  const int sc = blockIdx.y;
  const int4 in = einfo[sc];
  const double alpha = salpha[sc];
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double e[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (alpha != 0.0) {
    if (j < in.y) tet_energy_delta(in.x + j, tets, Dminv, vol, mu_, lam_, x, d, alpha, h2, e);
    if (j < in.w) vertex_energy_delta(in.z + j, mass, x, d, alpha, xtilde, h2, gx, gy, gz, hs, e);
  }
  block_sum<5>(e);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) part[5 * (int64_t(sc) * gridDim.x + blockIdx.x) + k] = e[k];
}

// x += alpha_s d with s the scene of the vertex (256-vertex blocks are
// single-scene).
__global__ void k_baxpy(int64_t n, const int32_t* __restrict__ ubscene, const double* __restrict__ salpha,
                        const double* __restrict__ d, double* __restrict__ x) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double a = salpha[ubscene[v / 256]];
  if (a == 0.0) return;
#pragma unroll
  for (int i = 0; i < 3; ++i) x[3 * v + i] += a * d[3 * v + i];
}

// Per-scene largest safe step toward the half-space (as k_ccd, over each
// scene's vertex range): block minima of min(1, safety dist / (-n.d)) over
// approaching vertices, then one block per scene takes the minimum of its
// partials.  Minima are exact, so each scene gets its unbatched value.
__global__ void __launch_bounds__(256) k_bccd(const int4* __restrict__ einfo, const double* __restrict__ x,
                                              const double* __restrict__ d, HalfSpace hs, double safety,
                                              double* __restrict__ part) {
  const int sc = blockIdx.y;
  const int4 in = einfo[sc];
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double a = 1.0;
  if (j < in.w) {
    const int64_t v = in.z + j;
    const double dist = hs.n[0] * x[3 * v] + hs.n[1] * x[3 * v + 1] + hs.n[2] * x[3 * v + 2] - hs.off;
    const double app = -(hs.n[0] * d[3 * v] + hs.n[1] * d[3 * v + 1] + hs.n[2] * d[3 * v + 2]);
    if (app > 0.0) a = fmin(a, safety * dist / app);
  }
  __shared__ double sh[4];
  a = wave_min(a);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sh[0];
    for (int w = 1; w < int(blockDim.x >> 6); ++w) m = fmin(m, sh[w]);
    part[int64_t(sc) * gridDim.x + blockIdx.x] = m;
  }
}

__global__ void k_bccd_finish(int nblk, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double m = 1.0;
  for (int b = 0; b < nblk; ++b) m = fmin(m, part[int64_t(blockIdx.x) * nblk + b]);
  out[8 * blockIdx.x] = m;
}

}  // namespace

void free_plan(BatchPlan* B) {
  if (!B) return;
  for (auto& row : B->graph)
    for (auto& g : row)
      if (g) (void)hipGraphExecDestroy(g);
  if (B->u) ms_destroy(B->u);
  delete B;
}

void destroy_batch(ms_ctx* c) {
  if (!c || !c->batch) return;
  free_plan(c->batch);
  c->batch = nullptr;
}

namespace {

ms_status build_plan(ms_ctx* const* scenes, int ns, BatchPlan*& out) {
  ms_ctx* c0 = scenes[0];
  auto* B = new BatchPlan();
  B->ns = ns;
  B->scenes.assign(scenes, scenes + ns);
  int64_t nv = 0, nt = 0;
  for (int s = 0; s < ns; ++s) {
    ms_ctx* c = scenes[s];
    B->n_s.push_back(c->n);
    B->T_s.push_back(c->T);
    B->v0.push_back(nv);
    B->t0.push_back(nt);
    const int64_t pad = ((c->n + 255) / 256) * 256;
    B->npad.push_back(pad);
    nv += pad;
    nt += c->T;
  }
  std::vector<double> rest(3 * nv, 0.0), E, nu, rho;
  std::vector<int32_t> tets;
  tets.reserve(4 * nt);
  for (int s = 0; s < ns; ++s) {
    ms_ctx* c = scenes[s];
    std::copy(c->h_rest.begin(), c->h_rest.end(), rest.begin() + 3 * B->v0[s]);
    for (int64_t q = 0; q < 4 * c->T; ++q) tets.push_back(int32_t(c->h_tets[q] + B->v0[s]));
    E.insert(E.end(), c->h_E.begin(), c->h_E.end());
    nu.insert(nu.end(), c->h_nu.begin(), c->h_nu.end());
    rho.insert(rho.end(), c->h_rho.begin(), c->h_rho.end());
  }
  ms_device dev = c0->dev;
  dev.hip_stream = c0->stream;
  ms_ctx* u = nullptr;
  ms_status st;
  if ((st = ms_create(&dev, &u))) {
    delete B;
    return fail(c0, st, "batch: context creation failed");
  }
  B->u = u;
  ms_ctx* const c = u;  // error reports of the HIP calls below
  if ((st = ms_upload_mesh(u, nv, rest.data(), nt, tets.data())) ||
      (st = ms_upload_material(u, E.data(), nu.data(), rho.data())) || (st = ms_set_gravity(u, c0->gravity)) ||
      (c0->has_hs && (st = ms_add_halfspace(u, c0->hs_n, c0->hs_off, c0->hs_dhat, c0->hs_kappa)))) {
    const std::string msg = "batch: union mesh: " + u->err;
    ms_destroy(u);
    delete B;
    return fail(c0, st, msg);
  }
  if (u->pat.S != c0->pat.S) {
    ms_destroy(u);
    delete B;
    return fail(c0, MS_E_ARG, "batch: scenes use another slice height than the union");
  }
  // segment maps
  const int64_t nbs = (u->pat.nslices + 3) / 4, nub = (nv + 255) / 256;
  B->nbs = nbs;
  B->nub = nub;
  std::vector<int32_t> tscene(nt), pbscene(nbs), ubscene(nub);
  std::vector<int4> sinfo(ns), einfo(ns);
  int64_t emax = 1;
  for (int s = 0; s < ns; ++s) {
    for (int64_t t = 0; t < B->T_s[s]; ++t) tscene[B->t0[s] + t] = s;
    const int64_t pb0 = B->v0[s] / 128, pbn = B->npad[s] / 128, ub0 = B->v0[s] / 256, ubn = B->npad[s] / 256;
    for (int64_t b = 0; b < pbn; ++b) pbscene[pb0 + b] = s;
    for (int64_t b = 0; b < ubn; ++b) ubscene[ub0 + b] = s;
    sinfo[s] = make_int4(int(pb0), int(pbn), int(ub0), int(ubn));
    einfo[s] = make_int4(int(B->t0[s]), int(B->T_s[s]), int(B->v0[s]), int(B->n_s[s]));
    emax = std::max<int64_t>(emax, (std::max(B->T_s[s], B->n_s[s]) + 255) / 256);
  }
  for (int64_t b = 0; b < nbs; ++b)  // product blocks past the last scene (none with aligned ranges)
    if (b * 128 >= nv) pbscene[b] = ns - 1;
  B->ebx = emax;
  const int64_t npart = std::max<int64_t>({3 * nbs, nub, 3 * ((3 * nv + 255) / 256), 5 * emax * ns});
  std::vector<int2> drange(ns), erange(ns);
  for (int s = 0; s < ns; ++s) {
    drange[s] = make_int2(int(3 * B->v0[s] / 256), int(3 * B->npad[s] / 256));
    erange[s] = make_int2(int(s * emax), int(emax));
  }
  if ((st = upload(u, &B->d_tscene, tscene.data(), tscene.size())) ||
      (st = upload(u, &B->d_pbscene, pbscene.data(), pbscene.size())) ||
      (st = upload(u, &B->d_ubscene, ubscene.data(), ubscene.size())) ||
      (st = upload(u, &B->d_sinfo, sinfo.data(), sinfo.size())) ||
      (st = upload(u, &B->d_einfo, einfo.data(), einfo.size())) ||
      (st = upload(u, &B->d_drange, drange.data(), drange.size())) ||
      (st = upload(u, &B->d_erange, erange.data(), erange.size())) ||
      (st = alloc_n(u, &B->d_sscal, size_t(kStride) * ns)) || (st = alloc_n(u, &B->d_sst, size_t(2 * ST_N) * ns)) ||
      (st = alloc_n(u, &B->d_salpha, size_t(ns))) || (st = alloc_n(u, &B->d_sproj, size_t(ns))) ||
      (st = alloc_n(u, &B->d_sactive, size_t(ns))) || (st = alloc_n(u, &B->d_sfirst, size_t(ns))) ||
      (st = alloc_n(u, &B->d_spart, size_t(npart))) || (st = alloc_n(u, &B->d_sout, size_t(8) * ns))) {
    const std::string msg = "batch: allocation: " + u->err;
    ms_destroy(u);
    delete B;
    return fail(c0, st, msg);
  }
  MS_HIP(hipMemsetAsync(B->d_sscal, 0, sizeof(double) * kStride * ns, u->stream));
  // padding vertices rest at the origin, at rest, massless (so without
  // contact terms) and pinned there
  MS_HIP(hipMemsetAsync(u->d_x, 0, sizeof(double) * 3 * u->n, u->stream));
  MS_HIP(hipMemsetAsync(u->d_v, 0, sizeof(double) * 3 * u->n, u->stream));
  B->h_sscal.assign(size_t(kStride) * ns, 0.0);
  out = B;
  return MS_OK;
}

// Segmented dots: (a0.b0, a1.b1, |a2 - am2|^2) per scene into h[8 s + k].
ms_status bdots(BatchPlan* B, const double* a0, const double* b0, const double* a1, const double* b1,
                const double* a2, const double* am2, std::vector<double>& h) {
  ms_ctx* u = B->u;
  ms_ctx* const c = u;
  const int64_t len = 3 * u->n;
  k_bdots<<<nblk(len, 256), 256, 0, u->stream>>>(len, a0, b0, a1, b1, a2, am2, B->d_spart);
  k_seg_finish<3><<<unsigned(B->ns), 256, 0, u->stream>>>(B->d_drange, B->d_spart, B->d_sout);
  h.resize(size_t(8) * B->ns);
  MS_HIP(hipMemcpyAsync(h.data(), B->d_sout, sizeof(double) * 8 * B->ns, hipMemcpyDeviceToHost, u->stream));
  return sync(u);
}

// Per-scene energy differences at the scene steps in d_salpha: h[8 s + k],
// k = 0..3 the parts, 4 the magnitude.
ms_status benergy(BatchPlan* B, const double* d, double h2, std::vector<double>& h) {
  ms_ctx* u = B->u;
  ms_ctx* const c = u;
  dim3 grid(unsigned(B->ebx), unsigned(B->ns));
  k_benergy_delta<<<grid, 256, 0, u->stream>>>(B->d_einfo, u->d_tets, u->d_Dminv, u->d_vol, u->d_mu, u->d_lam,
                                               u->d_mass, u->d_x, d, B->d_salpha, u->d_xtilde, h2, u->gravity[0],
                                               u->gravity[1], u->gravity[2], hs_of(u), B->d_spart);
  k_seg_finish<5><<<unsigned(B->ns), 256, 0, u->stream>>>(B->d_erange, B->d_spart, B->d_sout);
  h.resize(size_t(8) * B->ns);
  MS_HIP(hipMemcpyAsync(h.data(), B->d_sout, sizeof(double) * 8 * B->ns, hipMemcpyDeviceToHost, u->stream));
  return sync(u);
}

// Per-scene contact filter of the step d: h[8 s] = min(1, CCD bound) of
// scene s (1 without a half-space).
ms_status bccd(BatchPlan* B, const double* d, std::vector<double>& h) {
  ms_ctx* u = B->u;
  ms_ctx* const c = u;
  h.assign(size_t(8) * B->ns, 1.0);
  if (!u->has_hs) return MS_OK;
  dim3 grid(unsigned(B->ebx), unsigned(B->ns));
  k_bccd<<<grid, 256, 0, u->stream>>>(B->d_einfo, u->d_x, d, hs_of(u), 0.9, B->d_spart);
  k_bccd_finish<<<unsigned(B->ns), 64, 0, u->stream>>>(int(B->ebx), B->d_spart, B->d_sout);
  MS_HIP(hipMemcpyAsync(h.data(), B->d_sout, sizeof(double) * 8 * B->ns, hipMemcpyDeviceToHost, u->stream));
  return sync(u);
}

// Union basis for the two-level preconditioner: the scenes' bases side by
// side (handles renumbered from each scene's first union handle), installed
// as transfer operators only, and the block table of the block-diagonal
// coarse GEMV.  Every scene needs an installed basis with the exact coarse
// matrix and the same slice layout inside the union as in its own context.
std::vector<const void*> two_level_key(const BatchPlan* B) {
  std::vector<const void*> key;
  for (ms_ctx* sc : B->scenes) {
    key.push_back(sc->d_Ainv);
    key.push_back(sc->d_Ainv32);
    key.push_back(reinterpret_cast<const void*>(intptr_t(sc->r) << 32 | intptr_t(sc->rp)));
  }
  return key;
}

ms_status prepare_two_level(BatchPlan* B) {
  if (B->tl_ready && two_level_key(B) == B->tl_key) return MS_OK;
  // (re)build: a scene's basis was installed again since the tables were made
  for (auto& row : B->graph)
    if (row[1]) {
      (void)hipGraphExecDestroy(row[1]);
      row[1] = nullptr;
    }
  B->tl_ready = false;
  ms_ctx* u = B->u;
  ms_ctx* c0 = B->scenes[0];
  const int ns = B->ns, S = u->pat.S;
  Basis UB;
  UB.vptr.assign(u->n + 1, 0);
  B->h0.assign(ns, 0);
  B->slot0.assign(ns, 0);
  B->moved.assign(ns, 0.0);
  int32_t m = 0;
  for (int q = 0; q < ns; ++q) {
    ms_ctx* sc = B->scenes[q];
    if (!sc->has_basis) return fail(c0, MS_E_ORDER, "two-level batch: scene " + std::to_string(q) + " has no basis");
    if (sc->coarse_mode != MS_COARSE_EXACT)
      return fail(c0, MS_E_ARG, "two-level batch: scene " + std::to_string(q) + " integrates by cubature");
    // the scene's slices are a contiguous run of the union's with the same widths
    if (sc->pat.S != S) return fail(c0, MS_E_ARG, "two-level batch: scenes with another slice height");
    const int64_t s0 = B->v0[q] / S;
    const int64_t off = u->pat.h_slice_base[s0];
    for (int64_t k = 0; k <= sc->pat.nslices; ++k)
      if (u->pat.h_slice_base[s0 + k] - off != sc->pat.h_slice_base[k])
        return fail(c0, MS_E_ARG, "two-level batch: scene " + std::to_string(q) + " has another slice layout");
    B->slot0[q] = off;
    B->h0[q] = m;
    const Basis& D = sc->basis;
    for (int i = 0; i < D.m; ++i)
      for (int d = 0; d < 3; ++d) UB.origins.push_back(D.origins[3 * i + d]);
    m += D.m;
  }
  UB.m = m;
  for (int64_t v = 0, q = 0; v < u->n; ++v) {
    while (q + 1 < ns && v >= B->v0[q + 1]) ++q;
    const int64_t lv = v - B->v0[q];
    ms_ctx* sc = B->scenes[q];
    const Basis& D = sc->basis;
    if (lv < sc->n)
      for (int64_t k = D.vptr[lv]; k < D.vptr[lv + 1]; ++k) {
        UB.vhandle.push_back(D.vhandle[k] + B->h0[q]);
        UB.vphi.push_back(D.vphi[k]);
      }
    UB.vptr[v + 1] = int64_t(UB.vhandle.size());
  }
  ms_status st = install_transfer(u, UB);
  if (st) return fail(c0, st, "two-level batch: " + u->err);
  std::vector<GemvSeg> seg[2];
  B->rmax = 0;
  for (int q = 0; q < ns; ++q) {
    ms_ctx* sc = B->scenes[q];
    B->rmax = std::max(B->rmax, sc->r);
    for (int row = 0; row < sc->r; row += kGemvRowsPerBlock)
      for (int k = 0; k < 2; ++k) {
        GemvSeg g{};
        g.A = k == 0 ? static_cast<const void*>(sc->d_Ainv) : static_cast<const void*>(sc->d_Ainv32);
        g.ld = sc->rp;
        g.r = sc->r;
        g.row0 = row;
        g.h0 = B->h0[q];
        g.scene = q;
        seg[k].push_back(g);
      }
  }
  B->nseg = int(seg[0].size());
  for (int k = 0; k < 2; ++k)
    if ((st = upload(u, &B->d_seg[k], seg[k].data(), seg[k].size()))) return fail(c0, st, "two-level batch: " + u->err);
  B->tl_key = two_level_key(B);
  B->tl_ready = true;
  return MS_OK;
}

// u += U A_s^-1 U^T r for every scene (the additive coarse correction).
void bcoarse_correction(BatchPlan* B, int prec) {
  ms_ctx* u = B->u;
  launch_restrict(u, u->d_r, nullptr, nullptr);
  launch_coarse_gemv_seg(u, prec, B->d_seg[prec == MS_PREC_MIXED ? 1 : 0], B->nseg, B->rmax, B->d_sscal, kStride);
  launch_prolong_add(u, u->d_u, nullptr);
}

// The coarse matrix of scene q from its segment of the union's Hessian, and
// its inverse: the scene context's own Galerkin lists and factorisation,
// run on the union's values and stream.
ms_status scene_coarse_rebuild(BatchPlan* B, int q, int prec, double h2) {
  ms_ctx* sc = B->scenes[q];
  ms_ctx* u = B->u;
  double* v64 = sc->d_vals;
  float* v32 = sc->d_vals32;
  hipStream_t st = sc->stream;
  const int64_t off = 9 * B->slot0[q];
  sc->d_vals = u->d_vals ? u->d_vals + off : nullptr;
  sc->d_vals32 = u->d_vals32 ? u->d_vals32 + off : nullptr;
  sc->stream = u->stream;
  ms_status s = launch_galerkin(sc, prec, sc->d_x, h2);
  if (!s) s = coarse_factor(sc);
  sc->d_vals = v64;
  sc->d_vals32 = v32;
  sc->stream = st;
  return s;
}

void bcg_iteration(BatchPlan* B, int prec, int parity, bool tl) {
  ms_ctx* u = B->u;
  const int64_t ns = u->pat.nslices;
  const double* st_in = B->d_sst + ST_N * B->ns * parity;
  double* st_out = B->d_sst + ST_N * B->ns * (1 - parity);
  with_slice(u->pat.S, [&](auto SS) {
    constexpr int S = decltype(SS)::value;
    if (prec == MS_PREC_FP64)
      k_bcg_spmv<double, S><<<unsigned(B->nbs), 256, 0, u->stream>>>(u->n, ns, u->pat.d_slice_base, u->pat.d_col,
                                                                     u->d_vals, u->d_u, u->d_w, u->d_r, u->d_pinned,
                                                                     B->d_pbscene, B->d_sscal, u->d_part);
    else
      k_bcg_spmv<float, S><<<unsigned(B->nbs), 256, 0, u->stream>>>(u->n, ns, u->pat.d_slice_base, u->pat.d_col,
                                                                    u->d_vals32, u->d_u, u->d_w, u->d_r, u->d_pinned,
                                                                    B->d_pbscene, B->d_sscal, u->d_part);
  });
  if (prec == MS_PREC_FP64)
    k_bcg_update<double><<<unsigned(B->nub), 256, 0, u->stream>>>(u->n, B->d_ubscene, B->d_sinfo, u->d_part, st_in,
                                                                  st_out, u->d_p, u->d_s, u->d_d, u->d_r, u->d_u,
                                                                  u->d_w, u->d_Dinv, B->d_sscal);
  else
    k_bcg_update<float><<<unsigned(B->nub), 256, 0, u->stream>>>(u->n, B->d_ubscene, B->d_sinfo, u->d_part, st_in,
                                                                 st_out, u->d_p, u->d_s, u->d_d, u->d_r, u->d_u,
                                                                 u->d_w, u->d_Dinv32, B->d_sscal);
  if (tl) bcoarse_correction(B, prec);
}

// PCG on every active scene at once; on return h_sscal holds each scene's
// scalars (S_ITER, S_DONE: 1 converged, 2 iteration cap, 3 loss of positive
// definiteness, 5 inactive).
ms_status bpcg(BatchPlan* B, int prec, const ms_solver_params& P, const std::vector<uint8_t>& active,
               const std::vector<uint8_t>& first, bool tl) {
  ms_ctx* u = B->u;
  ms_ctx* const c = u;
  MS_HIP(hipMemcpyAsync(B->d_sactive, active.data(), active.size(), hipMemcpyHostToDevice, u->stream));
  MS_HIP(hipMemcpyAsync(B->d_sfirst, first.data(), first.size(), hipMemcpyHostToDevice, u->stream));
  if (prec == MS_PREC_FP64)
    k_bcg_init<double><<<unsigned(B->nub), 256, 0, u->stream>>>(u->n, u->d_g, u->d_pinned, u->d_p, u->d_s, u->d_d,
                                                                u->d_r, u->d_u, u->d_Dinv, B->d_spart);
  else
    k_bcg_init<float><<<unsigned(B->nub), 256, 0, u->stream>>>(u->n, u->d_g, u->d_pinned, u->d_p, u->d_s, u->d_d,
                                                               u->d_r, u->d_u, u->d_Dinv32, B->d_spart);
  k_bcg_init_finish<<<unsigned(B->ns), 256, 0, u->stream>>>(B->d_sinfo, B->d_spart, B->d_sactive, B->d_sfirst,
                                                            P.pcg_eta_max, P.pcg_eta_min, P.forcing,
                                                            double(P.max_pcg), B->d_sst, B->d_sscal);
  if (tl) bcoarse_correction(B, prec);  // u = S r + U A^-1 U^T r
  const int chunk = u->cg_chunk;
  hipGraphExec_t& ge = B->graph[prec == MS_PREC_FP64 ? 0 : 1][tl ? 1 : 0];
  if (!ge && u->use_graphs) {
    hipGraph_t g;
    MS_HIP(hipStreamBeginCapture(u->stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < chunk; ++i) bcg_iteration(B, prec, i & 1, tl);
    MS_HIP(hipStreamEndCapture(u->stream, &g));
    MS_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
  }
  int launched = 0;
  while (true) {
    if (u->use_graphs) {
      MS_HIP(hipGraphLaunch(ge, u->stream));
    } else {
      for (int i = 0; i < chunk; ++i) bcg_iteration(B, prec, i & 1, tl);
    }
    launched += chunk;
    MS_HIP(hipMemcpyAsync(B->h_sscal.data(), B->d_sscal, sizeof(double) * B->h_sscal.size(), hipMemcpyDeviceToHost,
                          u->stream));
    ms_status s = sync(u);
    if (s) return s;
    bool all = true;
    for (int q = 0; q < B->ns; ++q) all = all && B->h_sscal[size_t(kStride) * q + S_DONE] != 0.0;
    if (all) break;
    if (launched > P.max_pcg + 2 * chunk) return fail(u, MS_E_DEVICE, "batched PCG flags never set");
  }
  return MS_OK;
}

ms_status batch_step(BatchPlan* B, double dt, const ms_solver_params& P, ms_step_stats* out) {
  ms_ctx* u = B->u;
  ms_ctx* const c = u;
  const int ns = B->ns;
  const double h2 = dt * dt;
  const int prec = P.precision == MS_PREC_MIXED ? MS_PREC_MIXED : MS_PREC_FP64;
  const int64_t n3 = 3 * u->n;
  const bool tl = P.preconditioner == MS_PC_TWO_LEVEL_ADDITIVE;
  std::vector<ms_step_stats> S(ns);
  for (auto& st : S) st.min_alpha = 1.0;
  std::vector<uint8_t> active(ns, 1), first(ns, 1), proj(ns, 1), endgame(ns, 0), done(ns, 0);
  std::vector<double> alpha(ns, 0.0), h, he;
  ms_status s = MS_OK;
  u->timing = false;
  launch_predict(u, dt);
  launch_apply_dbc(u, int64_t(u->h_dbc.size()));
  if (P.predictor == 1) {  // inertial start, kept per scene where it lowers E
    launch_predictor_dir(u);
    if ((s = bccd(B, u->d_d, he))) return s;
    for (int q = 0; q < ns; ++q) alpha[q] = std::fmin(1.0, he[8 * q]);
    MS_HIP(hipMemcpyAsync(B->d_salpha, alpha.data(), sizeof(double) * ns, hipMemcpyHostToDevice, u->stream));
    if ((s = benergy(B, u->d_d, h2, he))) return s;
    for (int q = 0; q < ns; ++q) {
      double dE = he[8 * q] + he[8 * q + 1] + he[8 * q + 2] + he[8 * q + 3];
      alpha[q] = (std::isfinite(dE) && dE < 0.0) ? alpha[q] : 0.0;
    }
    MS_HIP(hipMemcpyAsync(B->d_salpha, alpha.data(), sizeof(double) * ns, hipMemcpyHostToDevice, u->stream));
    k_baxpy<<<nblk(u->n, 256), 256, 0, u->stream>>>(u->n, B->d_ubscene, B->d_salpha, u->d_d, u->d_x);
  }
  std::vector<double> dnorm(ns, 0.0), disp(ns, 0.0), xres(ns, 0.0);
  if ((s = bdots(B, nullptr, nullptr, u->d_x, u->d_x, nullptr, nullptr, h))) return s;
  for (int q = 0; q < ns; ++q) xres[q] = 1e-13 * std::sqrt(h[8 * q + 1]);
  for (int it = 0; it < P.max_newton; ++it) {
    bool any = false;
    for (int q = 0; q < ns; ++q) any = any || active[q];
    if (!any) break;
    for (int q = 0; q < ns; ++q) proj[q] = !(P.exact_endgame && endgame[q]);
    MS_HIP(hipMemcpyAsync(B->d_sproj, proj.data(), ns, hipMemcpyHostToDevice, u->stream));
    launch_element(u, u->d_x, h2, prec, true, true, B->d_tscene, B->d_sproj);
    launch_gather_grad(u, u->d_x, h2, u->d_g);
    launch_gather_hess(u, u->d_x, h2, prec);
    launch_block_jacobi(u, prec);
    u->assembled[prec == MS_PREC_FP64 ? 0 : 1] = true;
    if (tl) {
      // each scene's coarse operator, on the rule of its unbatched step:
      // at the first iteration, then after it has moved coarse_move x its
      // displacement (or every coarse_every iterations)
      for (int q = 0; q < ns && !s; ++q) {
        if (!active[q]) continue;
        bool refresh = it == 0;
        if (P.coarse_move > 0.0)
          refresh = refresh || B->moved[q] > P.coarse_move * std::max(disp[q], P.abs_floor);
        else
          refresh = refresh || (P.coarse_every > 0 && it % P.coarse_every == 0);
        if (!refresh) continue;
        B->moved[q] = 0.0;
        ++S[q].hessian_refreshes;
        s = scene_coarse_rebuild(B, q, prec, h2);
      }
      if (s) break;
    }
    if ((s = bpcg(B, prec, P, active, first, tl))) break;
    std::vector<uint8_t> step(ns, 0);
    for (int q = 0; q < ns; ++q) {
      if (!active[q]) continue;
      const double* sc = &B->h_sscal[size_t(kStride) * q];
      const int its = int(sc[S_ITER]), code = int(sc[S_DONE]);
      first[q] = 0;
      S[q].pcg_iters += its;
      S[q].max_pcg_iters = std::max(S[q].max_pcg_iters, its);
      if (!std::isfinite(sc[S_RHO0])) {
        s = fail(u, MS_E_NONFINITE, "non-finite gradient in scene " + std::to_string(q));
        break;
      }
      if (code == 3 && !proj[q]) {
        endgame[q] = 0;  // indefinite exact Hessian: this scene redoes the iteration projected
        continue;
      }
      step[q] = 1;
    }
    if (s) break;
    if ((s = bdots(B, u->d_g, u->d_d, u->d_d, u->d_d, nullptr, nullptr, h))) break;
    std::vector<double> gd(ns, 0.0);
    for (int q = 0; q < ns; ++q) {
      if (!step[q]) continue;
      gd[q] = h[8 * q];
      dnorm[q] = std::sqrt(h[8 * q + 1]);
      if (!std::isfinite(gd[q]) || !std::isfinite(dnorm[q])) {
        s = fail(u, MS_E_NONFINITE, "non-finite step in scene " + std::to_string(q));
        break;
      }
      if (dnorm[q] == 0.0) {
        step[q] = 0;
        active[q] = 0;
        done[q] = 1;
        S[q].newton_iters = it;
        continue;
      }
      if (!(gd[q] < 0.0)) {
        step[q] = 0;
        if (!proj[q]) {
          endgame[q] = 0;
          continue;
        }
        s = fail(u, MS_E_LINESEARCH, "search direction is not a descent direction in scene " + std::to_string(q));
        break;
      }
    }
    if (s) break;
    // line search, every stepping scene at its own alpha, from the CCD bound
    std::vector<uint8_t> searching(step);
    std::vector<int> nbt(ns, 0);
    if ((s = bccd(B, u->d_d, he))) break;
    for (int q = 0; q < ns; ++q) alpha[q] = step[q] ? std::fmin(1.0, he[8 * q]) : 0.0;
    while (true) {
      bool any_search = false;
      for (int q = 0; q < ns; ++q) any_search = any_search || searching[q];
      if (!any_search) break;
      std::vector<double> trial(ns, 0.0);
      for (int q = 0; q < ns; ++q) trial[q] = searching[q] ? alpha[q] : 0.0;
      MS_HIP(hipMemcpyAsync(B->d_salpha, trial.data(), sizeof(double) * ns, hipMemcpyHostToDevice, u->stream));
      if ((s = benergy(B, u->d_d, h2, he))) break;
      for (int q = 0; q < ns; ++q) {
        if (!searching[q]) continue;
        const double dE = he[8 * q] + he[8 * q + 1] + he[8 * q + 2] + he[8 * q + 3], err = he[8 * q + 4];
        if (std::isfinite(dE) && dE <= 1e-4 * alpha[q] * gd[q] + 1e-14 * err) {
          searching[q] = 0;
        } else {
          alpha[q] *= 0.5;
          if (++nbt[q] > P.max_backtracks) {
            s = fail(u, MS_E_LINESEARCH, "no energy decrease in scene " + std::to_string(q));
            break;
          }
        }
      }
      if (s) break;
    }
    if (s) break;
    MS_HIP(hipMemcpyAsync(B->d_salpha, alpha.data(), sizeof(double) * ns, hipMemcpyHostToDevice, u->stream));
    k_baxpy<<<nblk(u->n, 256), 256, 0, u->stream>>>(u->n, B->d_ubscene, B->d_salpha, u->d_d, u->d_x);
    if ((s = bdots(B, nullptr, nullptr, nullptr, nullptr, u->d_x, u->d_xt, h))) break;
    for (int q = 0; q < ns; ++q) {
      if (!step[q]) continue;
      S[q].backtracks += nbt[q];
      S[q].min_alpha = std::min(S[q].min_alpha, alpha[q]);
      if (tl) B->moved[q] += alpha[q] * dnorm[q];
      disp[q] = std::sqrt(h[8 * q + 2]);
      const double ref = std::max(disp[q], P.abs_floor);
      if (alpha[q] == 1.0 && (dnorm[q] <= P.newton_tol * ref || dnorm[q] <= xres[q])) {
        active[q] = 0;
        done[q] = 1;
        S[q].newton_iters = it + 1;
      } else if (dnorm[q] <= P.endgame_ratio * ref) {
        endgame[q] = 1;
      }
    }
  }
  bool all_done = !s;
  for (int q = 0; q < ns && all_done; ++q) all_done = done[q] != 0;
  if (!s && !all_done) s = fail(u, MS_E_NOCONV, "Newton did not converge in every scene");
  if (s) {
    (void)hipMemcpyAsync(u->d_x, u->d_xt, n3 * sizeof(double), hipMemcpyDeviceToDevice, u->stream);
    (void)hipStreamSynchronize(u->stream);
    return s;
  }
  launch_velocity(u, 1.0 / dt);
  if ((s = bdots(B, nullptr, nullptr, nullptr, nullptr, u->d_x, u->d_xt, h))) return s;
  for (int q = 0; q < ns; ++q) {
    S[q].last_dnorm = dnorm[q];
    S[q].disp_norm = std::sqrt(h[8 * q + 2]);
  }
  if (out)
    for (int q = 0; q < ns; ++q) out[q] = S[q];
  return MS_OK;
}

}  // namespace

}  // namespace ms

using namespace ms;

namespace ms {
namespace {

// The parameters a batched step supports.
ms_status batch_params(ms_ctx* c0, double dt, const ms_solver_params* pin, ms_solver_params& P) {
  if (!(dt > 0) || !std::isfinite(dt)) return fail(c0, MS_E_ARG, "dt must be positive");
  if (pin)
    P = *pin;
  else
    ms_solver_defaults(&P);
  if (P.mode != MS_MODE_PLAIN || P.warm_start || P.integrator != 0 ||
      (P.preconditioner != MS_PC_BLOCK_JACOBI && P.preconditioner != MS_PC_TWO_LEVEL_ADDITIVE))
    return fail(c0, MS_E_ARG,
                "batched steps support plain implicit-Euler mode with block-Jacobi or additive two-level PCG");
  if (P.precision == MS_PREC_MIXED && P.mixed_endgame_fp64)
    return fail(c0, MS_E_ARG, "batched steps keep one Hessian precision per step (no FP64 endgame)");
  if (P.smoother != 0) return fail(c0, MS_E_ARG, "batched steps smooth with 3x3 vertex blocks (smoother 0)");
  return MS_OK;
}

// Scenes a batch can hold: states set, one shared half-space or none, no
// friction, no self-contact, one device, one gravity, no repeats.
ms_status batch_scenes_ok(ms_ctx* const* scenes, int n_scenes) {
  ms_ctx* c0 = scenes[0];
  for (int q = 0; q < n_scenes; ++q) {
    ms_ctx* sc = scenes[q];
    if (sc->stage < 3) return fail(c0, MS_E_ORDER, "scene " + std::to_string(q) + " has no state");
    if (sc->has_hs != c0->has_hs) return fail(c0, MS_E_ARG, "scenes with and without a half-space");
    if (sc->has_hs) {
      bool same = sc->hs_off == c0->hs_off && sc->hs_dhat == c0->hs_dhat && sc->hs_kappa == c0->hs_kappa;
      for (int i = 0; i < 3; ++i) same = same && sc->hs_n[i] == c0->hs_n[i];
      if (!same) return fail(c0, MS_E_ARG, "scenes with different half-spaces");
      if (sc->hs_mu > 0.0) return fail(c0, MS_E_ARG, "batched steps do not support friction");
    }
    if (sc->sc.on) return fail(c0, MS_E_ARG, "batched steps do not support self-contact");
    if (sc->dev.device != c0->dev.device) return fail(c0, MS_E_ARG, "scenes on different devices");
    for (int i = 0; i < 3; ++i)
      if (sc->gravity[i] != c0->gravity[i]) return fail(c0, MS_E_ARG, "scenes with different gravity");
    for (int r = 0; r < q; ++r)
      if (scenes[r] == sc) return fail(c0, MS_E_ARG, "a scene appears twice");
  }
  return MS_OK;
}

// One batched timestep of the scenes on the union plan B.
ms_status batch_run(ms_ctx* const* scenes, int n_scenes, BatchPlan* B, double dt, const ms_solver_params& P,
                    ms_step_stats* per_scene) {
  ms_ctx* c0 = scenes[0];
  ms_ctx* u = B->u;
  ms_ctx* const c = u;
  // Dirichlet vertices of every scene plus the padding vertices, pinned
  std::vector<int32_t> dv;
  std::vector<double> dt3;
  for (int q = 0; q < n_scenes; ++q) {
    ms_ctx* sc = scenes[q];
    for (size_t k = 0; k < sc->h_dbc.size(); ++k) {
      dv.push_back(int32_t(sc->h_dbc[k] + B->v0[q]));
      for (int i = 0; i < 3; ++i) dt3.push_back(sc->h_dbc_tgt[3 * k + i]);
    }
    for (int64_t v = sc->n; v < B->npad[q]; ++v) {
      dv.push_back(int32_t(B->v0[q] + v));
      for (int i = 0; i < 3; ++i) dt3.push_back(0.0);
    }
  }
  ms_status s = ms_set_dirichlet(u, int64_t(dv.size()), dv.data(), dt3.data());
  if (s) return fail(c0, s, "batch: " + u->err);
  // states in
  for (int q = 0; q < n_scenes; ++q) {
    ms_ctx* sc = scenes[q];
    if (sc->stream != u->stream) MS_HIP(hipStreamSynchronize(sc->stream));
    MS_HIP(hipMemcpyAsync(u->d_x + 3 * B->v0[q], sc->d_x, 3 * sc->n * sizeof(double), hipMemcpyDeviceToDevice,
                          u->stream));
    MS_HIP(hipMemcpyAsync(u->d_v + 3 * B->v0[q], sc->d_v, 3 * sc->n * sizeof(double), hipMemcpyDeviceToDevice,
                          u->stream));
  }
  u->stage = 3;
  for (int q = 0; q < n_scenes; ++q) scenes[q]->has_prev = false;  // no BDF2 history across batched steps
  if (P.preconditioner == MS_PC_TWO_LEVEL_ADDITIVE) {
    if ((s = prepare_two_level(B))) return s;
    for (int q = 0; q < n_scenes; ++q) set_coarse_f32(scenes[q], P.precision == MS_PREC_MIXED);
  }
  s = batch_step(B, dt, P, per_scene);
  if (s) return fail(c0, s, "batch: " + u->err);
  for (int q = 0; q < n_scenes; ++q) {
    ms_ctx* sc = scenes[q];
    MS_HIP(hipMemcpyAsync(sc->d_x, u->d_x + 3 * B->v0[q], 3 * sc->n * sizeof(double), hipMemcpyDeviceToDevice,
                          u->stream));
    MS_HIP(hipMemcpyAsync(sc->d_v, u->d_v + 3 * B->v0[q], 3 * sc->n * sizeof(double), hipMemcpyDeviceToDevice,
                          u->stream));
  }
  return sync(u);
}

}  // namespace
}  // namespace ms

struct ms_batch {
  std::vector<ms_ctx*> scenes;
  BatchPlan* plan = nullptr;
};

extern "C" ms_status ms_batch_step(ms_ctx* const* scenes, int32_t n_scenes, double dt, const ms_solver_params* pin,
                                   ms_step_stats* per_scene) {
  if (!scenes || n_scenes < 1) return MS_E_ARG;
  for (int q = 0; q < n_scenes; ++q)
    if (!scenes[q]) return MS_E_ARG;
  ms_ctx* c0 = scenes[0];
  ms_solver_params P;
  ms_status s;
  if ((s = batch_params(c0, dt, pin, P)) || (s = batch_scenes_ok(scenes, n_scenes))) return s;
  // reuse the cached union when the scene list is unchanged
  BatchPlan* B = c0->batch;
  bool same = B && B->ns == n_scenes;
  for (int q = 0; same && q < n_scenes; ++q)
    same = B->scenes[q] == scenes[q] && B->n_s[q] == scenes[q]->n && B->T_s[q] == scenes[q]->T;
  if (!same) {
    destroy_batch(c0);
    BatchPlan* nb = nullptr;
    if ((s = build_plan(scenes, n_scenes, nb))) return s;
    c0->batch = B = nb;
  }
  return batch_run(scenes, n_scenes, B, dt, P, per_scene);
}

extern "C" ms_status ms_batch_create(ms_ctx* const* scenes, int32_t n_scenes, ms_batch** out) {
  if (!scenes || n_scenes < 1 || !out) return MS_E_ARG;
  *out = nullptr;
  for (int q = 0; q < n_scenes; ++q)
    if (!scenes[q]) return MS_E_ARG;
  ms_status s = batch_scenes_ok(scenes, n_scenes);
  if (s) return s;
  BatchPlan* B = nullptr;
  if ((s = build_plan(scenes, n_scenes, B))) return s;
  auto* b = new ms_batch();
  b->scenes.assign(scenes, scenes + n_scenes);
  b->plan = B;
  *out = b;
  return MS_OK;
}

extern "C" ms_status ms_batch_advance(ms_batch* b, double dt, const ms_solver_params* pin,
                                      ms_step_stats* per_scene) {
  if (!b || b->scenes.empty()) return MS_E_ARG;
  const int ns = int(b->scenes.size());
  ms_ctx* c0 = b->scenes[0];
  ms_solver_params P;
  ms_status s;
  if ((s = batch_params(c0, dt, pin, P)) || (s = batch_scenes_ok(b->scenes.data(), ns))) return s;
  for (int q = 0; q < ns; ++q)
    if (b->plan->n_s[q] != b->scenes[q]->n || b->plan->T_s[q] != b->scenes[q]->T)
      return fail(c0, MS_E_ORDER, "scene " + std::to_string(q) + " changed since ms_batch_create");
  return batch_run(b->scenes.data(), ns, b->plan, dt, P, per_scene);
}

extern "C" void ms_batch_destroy(ms_batch* b) {
  if (!b) return;
  ms::free_plan(b->plan);
  delete b;
}
