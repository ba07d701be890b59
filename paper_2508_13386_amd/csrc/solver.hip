// Plain Newton-PCG timestep (Sec. 3.1).
//
// Per Newton iteration: element kernel + atomic-free gathers assemble g
// (FP64) and H (FP64 or FP32) at x; PCG (block-Jacobi or two-level) solves
// H d = -g to the forcing tolerance eta = min(eta_max, sqrt(||g|| / ||g_0||));
// the step is truncated by the contact filters (the half-space bound and the
// additive CCD of the self-contact pairs) and backtracked until the
// Armijo condition holds on the FP64 energy difference (evaluated term by
// term, with a round-off allowance).  The iteration stops after a
// full step with ||d|| <= newton_tol * max(||x - x^t||, abs_floor) or with
// ||d|| below the round-off resolution 1e-13 ||x|| of the positions.
//
// Near the minimiser the element Hessians are used without the PSD
// projection (the exact Hessian), which restores quadratic convergence;
// if PCG then detects a loss of positive definiteness the iteration is
// redone with the projection.  A failed step restores x (transactional).
#include <chrono>
#include <cmath>
#include <cstdio>

#include "ms_internal.h"

namespace ms {

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static ms_status restore(ms_ctx* c, ms_status s) {
  (void)hipMemcpyAsync(c->d_x, c->d_xt, 3 * c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  (void)hipStreamSynchronize(c->stream);
  return s;
}

// Backtracking line search along d from x; returns the accepted alpha.
// The Armijo test uses the energy difference computed term by term (no
// cancellation of the large totals), with an allowance of 1e-14 times the
// magnitude of its terms for round-off.
ms_status line_search(ms_ctx* c, double h2, double gd, int max_bt, double* alpha_out, int* nbt) {
  double alpha = 1.0;
  ms_status s;
  if (c->has_hs) {
    launch_ccd(c, c->d_x, c->d_d);
    if ((s = read_scal(c))) return s;
    alpha = std::fmin(1.0, c->h_scal[S_CCD]);
  }
  if (c->sc.on) {
    double t;
    if ((s = sc_ccd(c, c->d_x, c->d_d, &t))) return s;
    alpha = std::fmin(alpha, t);
  }
  int k = 0;
  while (true) {
    double dE, err;
    if ((s = energy_delta(c, c->d_x, c->d_d, alpha, h2, &dE, &err))) return s;
    if (std::isfinite(dE) && dE <= 1e-4 * alpha * gd + 1e-14 * err) break;
    alpha *= 0.5;
    if (++k > max_bt) return fail(c, MS_E_LINESEARCH, "no energy decrease within the backtracking budget");
  }
  *alpha_out = alpha;
  *nbt = k;
  return MS_OK;
}

// Initial iterate from the inertial predictor: d = x~ - x on the free
// vertices (zero on Dirichlet ones), truncated by the contact filter; the
// move is kept only if it lowers the energy.
ms_status inertial_start(ms_ctx* c, double h2) {
  launch_predictor_dir(c);  // d = x~ - x, zero on pinned vertices
  return try_move(c, h2);
}

// x <- x + alpha d with alpha from the contact filter when E decreases.
ms_status try_move(ms_ctx* c, double h2) {
  ms_status s;
  double alpha = 1.0;
  if (c->has_hs) {
    launch_ccd(c, c->d_x, c->d_d);
    if ((s = read_scal(c))) return s;
    alpha = std::fmin(1.0, c->h_scal[S_CCD]);
  }
  if (c->sc.on) {
    double t;
    if ((s = sc_ccd(c, c->d_x, c->d_d, &t))) return s;
    alpha = std::fmin(alpha, t);
  }
  double dE, err;
  if ((s = energy_delta(c, c->d_x, c->d_d, alpha, h2, &dE, &err))) return s;
  if (std::isfinite(dE) && dE < 0.0) launch_axpy(c, c->d_x, c->d_d, alpha, 3 * c->n);
  return MS_OK;
}

ms_status plain_step(ms_ctx* c, double dt, const ms_solver_params& P, ms_step_stats* st) {
  const double t0 = now_ms();
  // BDF2 once a previous step is known (the first step is implicit Euler)
  const bool bdf2 = P.integrator == 1 && c->has_prev;
  const double h2 = (bdf2 ? 4.0 / 9.0 : 1.0) * dt * dt;
  int prec = P.precision == MS_PREC_MIXED ? MS_PREC_MIXED : MS_PREC_FP64;
  set_coarse_f32(c, prec == MS_PREC_MIXED);
  const int pc = (P.preconditioner >= 0 && P.preconditioner <= 3) ? P.preconditioner : MS_PC_BLOCK_JACOBI;
  if (two_level(pc) && !c->has_basis) return fail(c, MS_E_ORDER, "two-level preconditioner needs a basis");
  if (bdf2)
    launch_predict_bdf2(c, dt);
  else
    launch_predict(c, dt);
  launch_apply_dbc(c, int64_t(c->h_dbc.size()));
  c->timing = P.time_kernels != 0;
  c->proj_mode = P.projection == 1 ? 1 : 0;
  c->smoother = P.smoother == 1 ? 1 : 0;
  struct ProjReset {  // the eval and batch paths keep the clamp and the 3x3 blocks
    ms_ctx* c;
    ~ProjReset() {
      c->proj_mode = 0;
      c->smoother = 0;
    }
  } proj_reset{c};
  if (c->smoother) {
    ms_status sa = build_aggregates(c);
    if (sa) return restore(c, sa);
  }
  ms_step_stats S{};
  S.min_alpha = 1.0;
  ms_status s;
  if (P.warm_start && c->mlp) {
    if ((s = warm_start(c, dt, P.predictor == 1, &S.warm_start_used))) return restore(c, s);
  } else if (P.predictor == 1) {
    if ((s = inertial_start(c, h2))) return restore(c, s);
  }
  // round-off resolution of the positions (the step cannot be resolved below it)
  launch_dots(c, nullptr, nullptr, c->d_x, c->d_x, nullptr, nullptr);
  if ((s = read_scal(c))) return restore(c, s);
  const double xres = 1e-13 * std::sqrt(c->h_scal[S_DOT1]);
  bool endgame = false, converged = false, first = true, escalated = false;
  double dnorm = 0.0, disp = 0.0, moved = 0.0;
  int it = 0;
  for (; it < P.max_newton; ++it) {
    const bool project = !(P.exact_endgame && endgame);
    // the smoothed (deflation) form needs the Galerkin operator of the
    // Hessian it is applied with; the additive form only needs an SPD one
    bool refresh = it == 0 || escalated || pc == MS_PC_TWO_LEVEL;
    if (P.coarse_move > 0.0)
      refresh = refresh || moved > P.coarse_move * std::max(disp, P.abs_floor);
    else
      refresh = refresh || (P.coarse_every > 0 && it % P.coarse_every == 0);
    if (refresh) {
      moved = 0.0;
      if (two_level(pc)) ++S.hessian_refreshes;
    }
    escalated = false;
    // mixed precision: the tight solves of the endgame use the FP64 Hessian
    const int prec_it = (prec == MS_PREC_MIXED && endgame && P.mixed_endgame_fp64) ? MS_PREC_FP64 : prec;
    if ((s = assemble(c, c->d_x, h2, prec_it, project, true, pc, refresh))) return restore(c, s);
    int iters = 0, code = 0;
    if ((s = sync(c))) return restore(c, s);  // the assembly's kernels are not PCG time
    const double tp = now_ms();
    if ((s = pcg_solve(c, prec_it, pc, P.pcg_eta_max, P.pcg_eta_min, first, P.max_pcg, &iters, &code, P.forcing)))
      return restore(c, s);
    S.pcg_ms += now_ms() - tp;
    first = false;
    S.pcg_iters += iters;
    if (prec_it == MS_PREC_FP64) {
      S.pcg_iters_fp64 += iters;
      ++S.pcg_solves_fp64;
    }
    S.max_pcg_iters = std::max(S.max_pcg_iters, iters);
    if (!std::isfinite(c->h_scal[S_RHO0])) return restore(c, fail(c, MS_E_NONFINITE, "non-finite gradient"));
    if (code == 3 && !project) {  // indefinite exact Hessian: redo with the projection
      endgame = false;
      continue;
    }
    launch_dots(c, c->d_g, c->d_d, c->d_d, c->d_d, nullptr, nullptr);
    if ((s = read_scal(c))) return restore(c, s);
    const double gd = c->h_scal[S_DOT0];
    dnorm = std::sqrt(c->h_scal[S_DOT1]);
    if (!std::isfinite(gd) || !std::isfinite(dnorm)) return restore(c, fail(c, MS_E_NONFINITE, "non-finite step"));
    if (dnorm == 0.0) {
      converged = true;
      break;
    }
    if (!(gd < 0.0)) {
      if (!project) {
        endgame = false;
        continue;
      }
      return restore(c, fail(c, MS_E_LINESEARCH, "search direction is not a descent direction"));
    }
    double alpha = 1.0;
    int nbt = 0;
    if ((s = line_search(c, h2, gd, P.max_backtracks, &alpha, &nbt))) return restore(c, s);
    launch_axpy(c, c->d_x, c->d_d, alpha, 3 * c->n);
    moved += alpha * dnorm;
    S.backtracks += nbt;
    S.min_alpha = std::min(S.min_alpha, alpha);
    launch_dots(c, nullptr, nullptr, nullptr, nullptr, c->d_x, c->d_xt);
    if ((s = read_scal(c))) return restore(c, s);
    disp = std::sqrt(c->h_scal[S_DOT2]);
    const double ref = std::max(disp, P.abs_floor);
    if (c->verbose)
      std::fprintf(stderr,
                   "[ms] it %d proj %d pcg %d code %d eta %.2e |g| %.3e gd %.3e |d| %.3e alpha %.3g bt %d disp %.3e\n",
                   it, int(project), iters, code, c->h_scal[S_ETA], std::sqrt(c->h_scal[S_RHO0]), gd, dnorm, alpha, nbt,
                   disp);
    if (alpha == 1.0 && (dnorm <= P.newton_tol * ref || dnorm <= xres)) {
      converged = true;
      ++it;
      break;
    }
    if (dnorm <= P.endgame_ratio * ref) endgame = true;
    // Mixed precision: a timestep that has not converged after
    // mixed_max_newton iterations (the FP32 Hessian can limit the
    // contraction on ill-conditioned systems) is finished in FP64, with the
    // FP64 coarse inverse too: rounded to FP32 the inverse of an
    // ill-conditioned coarse matrix can lose positive definiteness, which
    // the continuation must not inherit.
    if (prec == MS_PREC_MIXED && P.mixed_max_newton > 0 && it + 1 >= P.mixed_max_newton) {
      prec = MS_PREC_FP64;
      escalated = true;
      set_coarse_f32(c, false);  // FP64 throughout, the coarse inverse included
      ++S.precision_escalations;
      if (c->verbose) std::fprintf(stderr, "[ms] it %d: continuing in FP64\n", it);
    }
  }
  if (!converged) return restore(c, fail(c, MS_E_NOCONV, "Newton did not converge"));
  // everything that can fail runs before v and the history change, so a
  // failure restores x and leaves v, x^{t-1}, v^{t-1} and q as they were
  double ef[4];
  if ((s = energy(c, c->d_x, nullptr, 0.0, h2, ef))) return restore(c, s);
  if (c->has_basis && c->mlp) {
    if ((s = record_coarse(c))) return restore(c, s);
  }
  launch_velocity_hist(c, dt, bdf2);
  c->has_prev = true;
  S.newton_iters = it;
  S.energy = ef[0] + ef[1] + ef[2] + ef[3];
  S.last_dnorm = dnorm;
  S.disp_norm = disp;
  S.time_ms = now_ms() - t0;
  if (st) *st = S;
  return MS_OK;
}

}  // namespace ms
