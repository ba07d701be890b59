// C ABI entry points: context lifetime, uploads, state, evaluation queries,
// and the plain Newton-PCG timestep (Sec. 3.1: x^{t+1} = argmin E, Newton
// steps H d = -g, CCD-filtered backtracking line search).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "ms_internal.h"

namespace ms {

ms_status fail(ms_ctx* c, ms_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}
ms_status hip_fail(ms_ctx* c, hipError_t e, const char* what) {
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return MS_E_DEVICE;
}
void* dalloc(ms_ctx* c, size_t bytes) {
  void* p = nullptr;
  if (c->dev.alloc) {
    p = c->dev.alloc(bytes, c->dev.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->allocs.push_back(p);
  return p;
}
void dfree(ms_ctx* c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c->allocs.size(); ++i)
    if (c->allocs[i] == p) {
      c->allocs[i] = c->allocs.back();
      c->allocs.pop_back();
      break;
    }
  if (c->dev.free)
    c->dev.free(p, c->dev.user);
  else
    (void)hipFree(p);
}
void release_all(ms_ctx* c) {
  (void)hipStreamSynchronize(c->stream);
  for (void* p : c->allocs) {
    if (c->dev.free)
      c->dev.free(p, c->dev.user);
    else
      (void)hipFree(p);
  }
  c->allocs.clear();
}

static bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

ms_status sync(ms_ctx* c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kernel execution");
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return MS_OK;
}

ms_status read_scal(ms_ctx* c) {
  hipError_t e = hipMemcpyAsync(c->h_scal, c->d_scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync scalars");
  return sync(c);
}

static ms_status alloc_workspace(ms_ctx* c) {
  const int64_t n = c->n, T = c->T, n3 = 3 * n;
  ms_status s;
  if ((s = alloc_n(c, &c->d_x, n3)) || (s = alloc_n(c, &c->d_v, n3)) || (s = alloc_n(c, &c->d_xt, n3)) ||
      (s = alloc_n(c, &c->d_xprev, n3)) || (s = alloc_n(c, &c->d_vprev, n3)) ||
      (s = alloc_n(c, &c->d_xtilde, n3)) || (s = alloc_n(c, &c->d_xtrial, n3)) || (s = alloc_n(c, &c->d_g, n3)) ||
      (s = alloc_n(c, &c->d_ge, 12 * T)) || (s = alloc_n(c, &c->d_He, 90 * T)) ||
      (s = alloc_n(c, &c->d_He32, 90 * T)) || (s = alloc_n(c, &c->d_vals, 9 * c->pat.nslots)) ||
      (s = alloc_n(c, &c->d_vals32, 9 * c->pat.nslots)) || (s = alloc_n(c, &c->d_Dinv, 9 * n)) ||
      (s = alloc_n(c, &c->d_Dinv32, 9 * n)) || (s = alloc_n(c, &c->d_d, n3)) || (s = alloc_n(c, &c->d_r, n3)) ||
      (s = alloc_n(c, &c->d_u, n3)) || (s = alloc_n(c, &c->d_w, n3)) || (s = alloc_n(c, &c->d_p, n3)) ||
      (s = alloc_n(c, &c->d_s, n3)) ||
      (s = alloc_n(c, &c->d_scal, S_COUNT)) || (s = alloc_n(c, &c->d_counter, 4)) ||
      (s = alloc_n(c, &c->d_cgst, 8)) ||
      (s = alloc_n(c, &c->d_pinned, n)))
    return s;
  const int64_t nparts = std::max<int64_t>(std::max(T, n3) / 64 + 64, 4096);
  if ((s = alloc_n(c, &c->d_part, 4 * nparts))) return s;
  MS_HIP(hipMemsetAsync(c->d_counter, 0, 16, c->stream));
  MS_HIP(hipMemsetAsync(c->d_scal, 0, S_COUNT * sizeof(double), c->stream));
  MS_HIP(hipMemsetAsync(c->d_vals, 0, 9 * c->pat.nslots * sizeof(double), c->stream));
  MS_HIP(hipMemsetAsync(c->d_vals32, 0, 9 * c->pat.nslots * sizeof(float), c->stream));
  MS_HIP(hipMemsetAsync(c->d_pinned, 0, n, c->stream));
  MS_HIP(hipMemsetAsync(c->d_v, 0, n3 * sizeof(double), c->stream));
  if (!c->h_scal) MS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_scal), S_COUNT * sizeof(double)));
  return sync(c);
}

static void destroy_graphs(ms_ctx* c) {
  for (auto& row : c->cg_graph)
    for (auto& g : row)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
}

void set_coarse_f32(ms_ctx* c, bool on) {
  if (c->coarse_f32 == on) return;
  for (auto& g : c->cg_graph[MS_PREC_FP64])
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  c->coarse_f32 = on;
}

// Runs PCG on H d = -g with the Hessian and preconditioner already built.
// Returns the device "done" code in *code (1 converged, 2 iteration cap,
// 3 loss of positive definiteness).
ms_status pcg_solve(ms_ctx* c, int prec, int pc, double eta_max, double eta_min, bool first, int max_it, int* iters,
                    int* code, int forcing) {
  launch_cg_init(c, prec, eta_max, eta_min, first, max_it, forcing);
  if (c->smoother) launch_agg_apply(c, prec);  // u = B^-1 r in place of the 3x3 blocks' S r
  if (pc == MS_PC_TWO_LEVEL) launch_coarse_start(c, prec);
  launch_precond_apply(c, prec, pc);
  if (c->cg_graph_smoother != c->smoother) {  // graphs hold the update kernel of one smoother
    destroy_graphs(c);
    c->cg_graph_smoother = c->smoother;
  }
  const int chunk = c->cg_chunk;
  hipGraphExec_t& ge = c->cg_graph[prec][pc];
  if (!ge && c->use_graphs) {
    hipGraph_t g;
    MS_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < chunk; ++i) launch_cg_iteration(c, prec, pc, i & 1);
    MS_HIP(hipStreamEndCapture(c->stream, &g));
    MS_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
  }
  int launched = 0;
  if (c->timing && int(c->tev.size()) < 2 * chunk) {
    c->tev.resize(2 * chunk, nullptr);
    for (auto& e : c->tev)
      if (!e) MS_HIP(hipEventCreate(&e));
  }
  while (true) {
    const int before = launched == 0 ? 0 : int(c->h_scal[S_ITER]);
    if (c->timing) {
      for (int i = 0; i < chunk; ++i) launch_cg_iteration(c, prec, pc, i & 1, c->tev[2 * i], c->tev[2 * i + 1]);
    } else if (c->use_graphs) {
      MS_HIP(hipGraphLaunch(ge, c->stream));
    } else {
      for (int i = 0; i < chunk; ++i) launch_cg_iteration(c, prec, pc, i & 1);
    }
    launched += chunk;
    ms_status s = read_scal(c);
    if (s) return s;
    if (c->timing) {
      // launches that ran a real iteration: those before convergence was flagged
      const int ran = std::min(chunk, int(c->h_scal[S_ITER]) - before + (c->h_scal[S_DONE] != 0.0 ? 1 : 0));
      for (int i = 0; i < std::max(0, ran); ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->tev[2 * i], c->tev[2 * i + 1]) == hipSuccess) {
          c->timed_ms[prec == MS_PREC_FP64 ? 0 : 1] += ms;
          c->timed_n[prec == MS_PREC_FP64 ? 0 : 1] += 1;
        }
      }
    }
    if (c->h_scal[S_DONE] != 0.0) break;
    if (launched > max_it + 2 * chunk) return fail(c, MS_E_DEVICE, "PCG flag never set");
  }
  *iters = int(c->h_scal[S_ITER]);
  *code = int(c->h_scal[S_DONE]);
  return MS_OK;
}

ms_status assemble(ms_ctx* c, const double* x, double h2, int prec, bool project, bool need_pc, int pc,
                   bool refresh_coarse) {
  c->assembled[prec == MS_PREC_FP64 ? 0 : 1] = true;
  c->asm_x = x;
  c->asm_h2 = h2;
  launch_element(c, x, h2, prec, true, project);
  launch_gather_grad(c, x, h2, c->d_g);
  launch_gather_hess(c, x, h2, prec);
  // the coarse matrix is formed before the self-contact terms join the
  // Hessian: it stays the (SPD) Galerkin operator of the rest
  if (need_pc && two_level(pc) && (refresh_coarse || !c->coarse_valid)) {
    ms_status s = launch_galerkin(c, prec, x, h2);
    if (s) return s;
    s = coarse_factor(c);
    if (s) return s;
  }
  if (c->sc.on) {
    ms_status s = sc_assemble(c, x, h2, prec);
    if (s) return s;
  }
  if (need_pc) {
    if (pc == MS_PC_TWO_LEVEL_VCYCLE)
      launch_block_jacobi_l1(c, prec);
    else
      launch_block_jacobi(c, prec);
    if (c->smoother) launch_agg_invert(c, prec);
  }
  return MS_OK;
}

ms_status energy_delta(ms_ctx* c, const double* x, const double* d, double alpha, double h2, double* dE,
                       double* err) {
  launch_energy_delta(c, x, d, alpha, h2);
  ms_status s = read_scal(c);
  if (s) return s;
  *dE = c->h_scal[S_DE0] + c->h_scal[S_DE1] + c->h_scal[S_DE2] + c->h_scal[S_DE3];
  *err = c->h_scal[S_DE4];
  if (c->sc.on) {
    double dc, ec;
    if ((s = sc_energy_delta(c, x, d, alpha, h2, &dc, &ec))) return s;
    *dE += dc;
    *err += ec;
  }
  return MS_OK;
}

ms_status energy(ms_ctx* c, const double* x, const double* d, double alpha, double h2, double parts[4]) {
  launch_energy(c, x, d, alpha, h2);
  ms_status s = read_scal(c);
  if (s) return s;
  for (int k = 0; k < 4; ++k) parts[k] = c->h_scal[S_E0 + k];
  if (c->sc.on) {
    const double* y = x;
    if (d) {
      launch_fill(c, c->sc.d_y, 0.0, 3 * c->n);
      launch_axpy(c, c->sc.d_y, x, 1.0, 3 * c->n);
      launch_axpy(c, c->sc.d_y, d, alpha, 3 * c->n);
      y = c->sc.d_y;
    }
    double e;
    if ((s = sc_energy(c, y, h2, &e))) return s;
    parts[3] += e;
  }
  return MS_OK;
}

}  // namespace ms

using namespace ms;

extern "C" {

void ms_solver_defaults(ms_solver_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->mode = MS_MODE_PLAIN;
  p->precision = MS_PREC_FP64;
  p->preconditioner = MS_PC_BLOCK_JACOBI;
  p->max_newton = 50;
  p->max_pcg = 20000;
  p->newton_tol = 1e-9;
  p->abs_floor = 1e-9;
  p->pcg_eta_max = 0.5;
  p->pcg_eta_min = 1e-12;
  p->max_backtracks = 30;
  p->exact_endgame = 1;
  p->warm_start = 0;
  p->paper_eps = 1e-3;
  p->subspace_rtol = 1e-4;
  p->refine_iters = 0;
  p->lag_window = 3;
  p->lag_threshold = 0.5;
  p->lag_min_gap = 5;
  p->forcing = 0;
  p->endgame_ratio = 1e-3;
  p->coarse_every = 1;
  p->predictor = 1;
  p->coarse_move = 0.0;
  p->mixed_max_newton = 20;
  p->mixed_endgame_fp64 = 0;
  p->integrator = 0;
  p->smoother = 0;
}

void ms_basis_defaults(ms_basis_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n_handles = 43;
  p->oversample = 1.5;
  p->jump_penalty = 0.25;
  p->prune_ratio = 1.75;
  p->prune_every = 10;
  p->prune_n = 5;
  p->max_lloyd = 50;
  p->lattice_seeding = 0;
  p->seed = 0;
  p->n_threads = 0;
  p->gpu_min_unknowns = 4096;
  p->rigid_contrast = 0.0;
}

ms_status ms_create(const ms_device* dev, ms_ctx** out) {
  if (!dev || !out) return MS_E_ARG;
  if (hipSetDevice(dev->device) != hipSuccess) return MS_E_DEVICE;
  ms_ctx* c = new ms_ctx();
  c->dev = *dev;
  if (const char* v = std::getenv("MS_VERBOSE")) c->verbose = std::atoi(v);
  // PCG launch configuration: iterations per captured graph (and per look
  // at the done flag; even, since iterations alternate two recurrence-state
  // buffers), and graphs or plain stream launches
  if (const char* v = std::getenv("MS_CG_CHUNK")) c->cg_chunk = std::min(256, std::max(2, std::atoi(v))) & ~1;
  if (const char* v = std::getenv("MS_CG_GRAPHS")) c->use_graphs = std::atoi(v) != 0;
  if (dev->hip_stream) {
    c->stream = static_cast<hipStream_t>(dev->hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return MS_E_DEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return MS_OK;
}

const char* ms_last_error(const ms_ctx* c) { return c ? c->err.c_str() : "null context"; }

ms_status ms_upload_mesh(ms_ctx* c, int64_t n, const double* rest, int64_t T, const int32_t* tets) {
  if (!c) return MS_E_ARG;
  if (c->stage >= 1) return fail(c, MS_E_ORDER, "mesh already uploaded");
  if (n < 4 || T < 1 || !rest || !tets) return fail(c, MS_E_ARG, "need n >= 4, T >= 1 and non-null arrays");
  if (n > (int64_t(1) << 30) || T > (int64_t(1) << 26)) return fail(c, MS_E_ARG, "mesh too large");
  if (!finite_all(rest, 3 * n)) return fail(c, MS_E_NONFINITE, "non-finite rest position");
  for (int64_t i = 0; i < 4 * T; ++i)
    if (tets[i] < 0 || tets[i] >= n) return fail(c, MS_E_ARG, "tet vertex index out of range");
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (tets[4 * t + a] == tets[4 * t + b]) return fail(c, MS_E_MESH, "tet with repeated vertex");
  c->n = n;
  c->T = T;
  c->h_rest.assign(rest, rest + 3 * n);
  c->h_tets.assign(tets, tets + 4 * T);
  ms_status s = build_mesh(c);
  if (s) return s;
  c->stage = 1;
  return MS_OK;
}

ms_status ms_upload_material(ms_ctx* c, const double* E, const double* nu, const double* rho) {
  if (!c) return MS_E_ARG;
  if (c->stage < 1) return fail(c, MS_E_ORDER, "upload the mesh first");
  if (!E || !nu || !rho) return fail(c, MS_E_ARG, "null material array");
  const int64_t T = c->T, n = c->n;
  c->h_mu.resize(T);
  c->h_lam.resize(T);
  c->h_E.assign(E, E + T);
  c->h_nu.assign(nu, nu + T);
  c->h_rho.assign(rho, rho + T);
  c->h_mass.assign(n, 0.0);
  for (int64_t t = 0; t < T; ++t) {
    if (!std::isfinite(E[t]) || !std::isfinite(nu[t]) || !std::isfinite(rho[t]))
      return fail(c, MS_E_NONFINITE, "non-finite material value");
    if (!(E[t] > 0) || !(nu[t] > -1.0 && nu[t] < 0.5) || !(rho[t] > 0))
      return fail(c, MS_E_ARG, "material out of range at tet " + std::to_string(t));
    const double mu = E[t] / (2.0 * (1.0 + nu[t]));
    const double lam = E[t] * nu[t] / ((1.0 + nu[t]) * (1.0 - 2.0 * nu[t]));
    c->h_mu[t] = mu;
    c->h_lam[t] = lam + mu;
    for (int a = 0; a < 4; ++a) c->h_mass[c->h_tets[4 * t + a]] += rho[t] * c->h_vol[t] / 4.0;
  }
  ms_status s;
  if ((s = upload(c, &c->d_mu, c->h_mu.data(), T))) return s;
  if ((s = upload(c, &c->d_lam, c->h_lam.data(), T))) return s;
  if ((s = upload(c, &c->d_mass, c->h_mass.data(), n))) return s;
  if (c->stage < 2) {
    if ((s = alloc_workspace(c))) return s;
    c->stage = 2;
  }
  return MS_OK;
}

ms_status ms_set_gravity(ms_ctx* c, const double g[3]) {
  if (!c || !g) return MS_E_ARG;
  if (!finite_all(g, 3)) return fail(c, MS_E_NONFINITE, "non-finite gravity");
  for (int i = 0; i < 3; ++i) c->gravity[i] = g[i];
  return MS_OK;
}

ms_status ms_set_dirichlet(ms_ctx* c, int64_t nd, const int32_t* verts, const double* tgt) {
  if (!c) return MS_E_ARG;
  if (c->stage < 2) return fail(c, MS_E_ORDER, "upload mesh and material first");
  if (nd < 0 || (nd > 0 && (!verts || !tgt))) return fail(c, MS_E_ARG, "bad Dirichlet arrays");
  if (!finite_all(tgt, 3 * nd)) return fail(c, MS_E_NONFINITE, "non-finite Dirichlet target");
  std::vector<uint8_t> pin(c->n, 0);
  for (int64_t i = 0; i < nd; ++i) {
    if (verts[i] < 0 || verts[i] >= c->n) return fail(c, MS_E_ARG, "Dirichlet vertex out of range");
    pin[verts[i]] = 1;
  }
  const bool same = (int64_t(c->h_dbc.size()) == nd) && std::equal(verts, verts + nd, c->h_dbc.begin());
  c->h_dbc.assign(verts, verts + nd);
  c->h_dbc_tgt.assign(tgt, tgt + 3 * nd);
  ms_status s;
  if (nd > c->dbc_cap) {
    if ((s = alloc_n(c, &c->d_dbc, nd)) || (s = alloc_n(c, &c->d_dbc_tgt, 3 * nd))) return s;
    c->dbc_cap = nd;
  }
  if (nd) {
    MS_HIP(hipMemcpyAsync(c->d_dbc, verts, nd * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    MS_HIP(hipMemcpyAsync(c->d_dbc_tgt, tgt, 3 * nd * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  MS_HIP(hipMemcpyAsync(c->d_pinned, pin.data(), c->n, hipMemcpyHostToDevice, c->stream));
  if (!same) c->coarse_valid = 0, c->cub.built = false;
  return sync(c);
}

ms_status ms_add_halfspace(ms_ctx* c, const double nrm[3], double off, double dhat, double kappa) {
  if (!c || !nrm) return MS_E_ARG;
  const double l = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
  if (!(l > 0) || !(dhat > 0) || !(kappa >= 0) || !std::isfinite(off) || !std::isfinite(l))
    return fail(c, MS_E_ARG, "bad half-space");
  for (int i = 0; i < 3; ++i) c->hs_n[i] = nrm[i] / l;
  c->hs_off = off / l;
  c->hs_dhat = dhat;
  c->hs_kappa = kappa;
  c->has_hs = true;
  return MS_OK;
}

ms_status ms_set_self_contact(ms_ctx* c, double dhat, double kappa, int32_t slots) {
  if (!c) return MS_E_ARG;
  if (c->stage != 1) return fail(c, MS_E_ORDER, "self-contact is set between ms_upload_mesh and ms_upload_material");
  if (!(dhat > 0.0) || !std::isfinite(dhat) || !(kappa > 0.0) || !std::isfinite(kappa) || slots < 1 || slots > 64)
    return fail(c, MS_E_ARG, "need dhat > 0, kappa > 0 and 1 <= slots <= 64");
  c->sc.on = true;
  c->sc.dhat = dhat;
  c->sc.kappa = kappa;
  c->sc.spare = slots;
  ms_status s = sc_setup(c);
  if (s) c->sc.on = false;
  return s;
}

ms_status ms_set_friction(ms_ctx* c, double mu, double eps_v) {
  if (!c) return MS_E_ARG;
  if (!c->has_hs) return fail(c, MS_E_ORDER, "add a half-space first");
  if (!(mu >= 0.0) || !std::isfinite(mu) || !(eps_v > 0.0) || !std::isfinite(eps_v))
    return fail(c, MS_E_ARG, "need mu >= 0 and eps_v > 0");
  c->hs_mu = mu;
  c->hs_epsv = eps_v;
  return MS_OK;
}

ms_status ms_set_state(ms_ctx* c, const double* x, const double* v) {
  if (!c) return MS_E_ARG;
  if (c->stage < 2) return fail(c, MS_E_ORDER, "upload mesh and material first");
  if (!x || !v) return fail(c, MS_E_ARG, "null state");
  const int64_t n3 = 3 * c->n;
  if (!finite_all(x, n3) || !finite_all(v, n3)) return fail(c, MS_E_NONFINITE, "non-finite state");
  if (c->has_hs)
    for (int64_t i = 0; i < c->n; ++i)
      if (c->hs_n[0] * x[3 * i] + c->hs_n[1] * x[3 * i + 1] + c->hs_n[2] * x[3 * i + 2] - c->hs_off <= 0.0)
        return fail(c, MS_E_ARG, "vertex outside the half-space");
  MS_HIP(hipMemcpyAsync(c->d_x, x, n3 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  MS_HIP(hipMemcpyAsync(c->d_v, v, n3 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  c->stage = 3;
  c->q_hist = 0;
  c->has_prev = false;
  return sync(c);
}

ms_status ms_get_state(const ms_ctx* cc, double* x, double* v) {
  ms_ctx* c = const_cast<ms_ctx*>(cc);
  if (!c) return MS_E_ARG;
  if (c->stage < 3) return fail(c, MS_E_ORDER, "no state");
  const int64_t n3 = 3 * c->n;
  if (x) MS_HIP(hipMemcpyAsync(x, c->d_x, n3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (v) MS_HIP(hipMemcpyAsync(v, c->d_v, n3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

ms_status ms_get_pattern(const ms_ctx* cc, int64_t* nnzb, int32_t* row_ptr, int32_t* col) {
  ms_ctx* c = const_cast<ms_ctx*>(cc);
  if (!c || !nnzb) return MS_E_ARG;
  if (c->stage < 1) return fail(c, MS_E_ORDER, "no mesh");
  *nnzb = c->pat.nnzb;
  if (row_ptr) std::memcpy(row_ptr, c->pat.h_row_ptr.data(), (c->n + 1) * sizeof(int32_t));
  if (col) std::memcpy(col, c->pat.h_col.data(), c->pat.nnzb * sizeof(int32_t));
  return MS_OK;
}

ms_status ms_eval(ms_ctx* c, const double* x, double dt, int32_t prec, double* e4, double* grad, double* hess) {
  if (!c || !x) return MS_E_ARG;
  if (c->stage < 3) return fail(c, MS_E_ORDER, "set a state first");
  if (prec != MS_PREC_FP64 && prec != MS_PREC_MIXED) return fail(c, MS_E_ARG, "bad precision");
  const int64_t n3 = 3 * c->n;
  if (!finite_all(x, n3)) return fail(c, MS_E_NONFINITE, "non-finite x");
  MS_HIP(hipMemcpyAsync(c->d_xtrial, x, n3 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  launch_predict(c, dt);
  const double h2 = dt * dt;
  ms_status s = assemble(c, c->d_xtrial, h2, prec, true, true, MS_PC_BLOCK_JACOBI, true);
  if (s) return s;
  if (c->has_basis) {
    if ((s = launch_galerkin(c, prec, c->d_xtrial, h2))) return s;
    if ((s = coarse_factor(c))) return s;
  }
  double parts[4];
  if ((s = energy(c, c->d_xtrial, nullptr, 0.0, h2, parts))) return s;
  if (e4) std::memcpy(e4, parts, sizeof(parts));
  if (grad) MS_HIP(hipMemcpyAsync(grad, c->d_g, n3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (hess) {
    // extract into the canonical BSR order through a temporary device buffer
    int64_t* d_slot = nullptr;
    double* d_out = nullptr;
    if ((s = upload(c, &d_slot, c->pat.h_slot_of_bsr.data(), c->pat.nnzb))) return s;
    if ((s = alloc_n(c, &d_out, 9 * c->pat.nnzb))) return s;
    launch_extract_bsr(c, d_slot, c->pat.nnzb, d_out, prec);
    MS_HIP(hipMemcpyAsync(hess, d_out, 9 * c->pat.nnzb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    s = sync(c);
    dfree(c, d_slot);
    dfree(c, d_out);
    if (s) return s;
  }
  c->eval_valid = true;
  c->eval_prec = prec;
  return sync(c);
}

ms_status ms_energy_difference(ms_ctx* c, const double* x, const double* d, double alpha, double dt,
                               double* parts5) {
  if (!c || !x || !d || !parts5 || !std::isfinite(alpha) || !(dt > 0)) return MS_E_ARG;
  if (c->stage < 3) return fail(c, MS_E_ORDER, "set a state first");
  const int64_t n3 = 3 * c->n;
  if (!finite_all(x, n3) || !finite_all(d, n3)) return fail(c, MS_E_NONFINITE, "non-finite x or d");
  MS_HIP(hipMemcpyAsync(c->d_xtrial, x, n3 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  MS_HIP(hipMemcpyAsync(c->d_w, d, n3 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  launch_predict(c, dt);
  launch_energy_delta(c, c->d_xtrial, c->d_w, alpha, dt * dt);
  ms_status s = read_scal(c);
  if (s) return s;
  for (int k = 0; k < 5; ++k) parts5[k] = c->h_scal[S_DE0 + k];
  if (c->sc.on) {
    double dc, ec;
    if ((s = sc_energy_delta(c, c->d_xtrial, c->d_w, alpha, dt * dt, &dc, &ec))) return s;
    parts5[3] += dc;
    parts5[4] += ec;
  }
  return MS_OK;
}

ms_status ms_apply_preconditioner(ms_ctx* c, int32_t kind, int32_t prec, const double* r, double* z) {
  if (!c || !r || !z) return MS_E_ARG;
  if (!c->eval_valid) return fail(c, MS_E_ORDER, "call ms_eval first");
  if (prec != c->eval_prec) return fail(c, MS_E_ARG, "precision differs from the last ms_eval");
  set_coarse_f32(c, false);
  if (kind < 0 || kind > 3) return fail(c, MS_E_ARG, "bad preconditioner kind");
  if (two_level(kind) && !c->has_basis) return fail(c, MS_E_ORDER, "no basis");
  if (kind == MS_PC_TWO_LEVEL && c->coarse_mode == MS_COARSE_CUBATURE)
    return fail(c, MS_E_ARG, "the smoothed two-level preconditioner needs the exact coarse matrix");
  const int64_t n3 = 3 * c->n;
  std::vector<double> mr(r, r + n3);
  for (auto& v : mr) v = -v;
  MS_HIP(hipMemcpyAsync(c->d_g, mr.data(), n3 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  // the V-cycle smooths with the l1-scaled inverses; ms_eval left the plain
  // block-Jacobi ones, restored afterwards
  if (kind == MS_PC_TWO_LEVEL_VCYCLE) launch_block_jacobi_l1(c, prec);
  launch_cg_init(c, prec, 0.0, 0.0, true, 0, 0);
  launch_precond_apply(c, prec, kind);
  if (kind == MS_PC_TWO_LEVEL_VCYCLE) launch_block_jacobi(c, prec);
  MS_HIP(hipMemcpyAsync(z, c->d_u, n3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

ms_status ms_step(ms_ctx* c, double dt, const ms_solver_params* pin, ms_step_stats* st) {
  if (!c) return MS_E_ARG;
  if (c->stage < 3) return fail(c, MS_E_ORDER, "set a state first");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(c, MS_E_ARG, "dt must be positive");
  ms_solver_params P;
  if (pin)
    P = *pin;
  else
    ms_solver_defaults(&P);
  if (!(P.coarse_move >= 0.0) || P.mixed_max_newton < 0)
    return fail(c, MS_E_ARG, "coarse_move and mixed_max_newton must not be negative");
  if (P.integrator != 0 && P.integrator != 1) return fail(c, MS_E_ARG, "integrator must be 0 or 1");
  if (P.projection != 0 && P.projection != 1) return fail(c, MS_E_ARG, "projection must be 0 or 1");
  if (P.smoother != 0 && P.smoother != 1) return fail(c, MS_E_ARG, "smoother must be 0 or 1");
  if (P.smoother == 1 && (P.mode != MS_MODE_PLAIN || c->sc.on ||
                          (P.preconditioner != MS_PC_BLOCK_JACOBI && P.preconditioner != MS_PC_TWO_LEVEL_ADDITIVE)))
    return fail(c, MS_E_ARG,
                "the aggregate smoother runs in plain mode with block-Jacobi or additive two-level PCG, "
                "without self-contact");
  if (P.integrator == 1 && P.mode == MS_MODE_PAPER) return fail(c, MS_E_ARG, "paper mode steps with implicit Euler");
  // the learned start is judged on the implicit Euler incremental potential
  if (P.integrator == 1 && P.warm_start && c->mlp)
    return fail(c, MS_E_ARG, "the learned warm start steps with implicit Euler");
  if (c->sc.on && P.mode == MS_MODE_PAPER) return fail(c, MS_E_ARG, "paper mode has no self-contact");
  if (c->sc.on && P.preconditioner == MS_PC_TWO_LEVEL)
    return fail(c, MS_E_ARG, "the smoothed two-level preconditioner has no self-contact");
  if (P.mode == MS_MODE_PAPER) return paper_step(c, dt, P, st);
  // the smoothed (deflated) form projects with the coarse matrix and stays a
  // symmetric positive definite preconditioner only for the exact U^T H U
  if (P.preconditioner == MS_PC_TWO_LEVEL && c->coarse_mode == MS_COARSE_CUBATURE)
    return fail(c, MS_E_ARG, "the smoothed two-level preconditioner needs the exact coarse matrix");
  return plain_step(c, dt, P, st);
}

void ms_destroy(ms_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  destroy_batch(c);
  destroy_mlp(c);
  destroy_graphs(c);
  for (auto& e : c->tev)
    if (e) (void)hipEventDestroy(e);
  release_all(c);
  if (c->h_scal) (void)hipHostFree(c->h_scal);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

ms_status ms_mat_create(const ms_device* dev, int64_t n, const int32_t* row_ptr, const int32_t* col,
                        const double* vals, int32_t dtype, ms_mat** out) {
  if (!dev || !out || !row_ptr || !col || !vals || n < 1 || (dtype != 0 && dtype != 1)) return MS_E_ARG;
  if (hipSetDevice(dev->device) != hipSuccess) return MS_E_DEVICE;
  ms_mat* A = new ms_mat();
  A->ctx.dev = *dev;
  A->ctx.stream = static_cast<hipStream_t>(dev->hip_stream);
  A->dtype = dtype;
  ms_status s = mat_build(A, n, row_ptr, col, vals);
  if (s) {
    ms_mat_destroy(A);
    return s;
  }
  *out = A;
  return MS_OK;
}
ms_status ms_mat_spmv(ms_mat* A, const void* x, void* y) {
  if (!A || !x || !y) return MS_E_ARG;
  mat_spmv(A, x, y);
  return hipGetLastError() == hipSuccess ? MS_OK : MS_E_DEVICE;
}
double ms_mat_bytes(const ms_mat* A) { return A ? A->bytes : 0.0; }

ms_status ms_time_kernel(ms_ctx* c, int32_t kernel, int32_t prec, int32_t reps, double* avg_us, double* bytes) {
  if (!c || !avg_us || !bytes || reps < 0 || kernel < 0 || kernel > 6 || (prec != MS_PREC_FP64 && prec != MS_PREC_MIXED))
    return MS_E_ARG;
  if (!c->assembled[prec == MS_PREC_FP64 ? 0 : 1]) return fail(c, MS_E_ORDER, "no Hessian assembled in that precision");
  if (reps == 0) {
    const int q = prec == MS_PREC_FP64 ? 0 : 1;
    if (c->timed_n[q] == 0) return fail(c, MS_E_ORDER, "no PCG products recorded");
    *avg_us = 1e3 * c->timed_ms[q] / double(c->timed_n[q]);
    *bytes = cg_spmv_bytes(c, prec);
    c->timed_ms[q] = 0.0;
    c->timed_n[q] = 0;
    return MS_OK;
  }
  if (kernel == 6) return time_coarse_matrix(c, prec, reps, avg_us, bytes);
  if (kernel > 0) {
    if (reps == 0) return fail(c, MS_E_ARG, "in-loop timing is recorded for kernel 0 only");
    return time_loop_kernel(c, kernel, prec, reps, avg_us, bytes);
  }
  return time_cg_spmv(c, prec, reps, avg_us, bytes);
}
void ms_mat_destroy(ms_mat* A) {
  if (!A) return;
  release_all(&A->ctx);
  delete A;
}

}  // extern "C"
