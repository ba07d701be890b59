// The paper's three-level inexact Newton timestep (Alg. 1 with the linear
// solves of Alg. 2).
//
// Per Newton iteration, with g and the PSD-projected Hessian H at x:
//   affine level     (U_a^T H U_a) q_a = -U_a^T g, d_s = U_a q_a; the 12x12
//                    system is formed from 12 lifted products H U_a e_k and
//                    solved exactly on the host (one block: block-Jacobi PCG
//                    on it converges in one iteration);
//   subspace level   (U_s^T H U_s) q_s = U_s^T r with r = -g - H d_s,
//                    d_s += U_s q_s, through the explicit inverse of the
//                    Galerkin matrix (an exact solve, tighter than the
//                    paper's relative residual of 1e-4);
//   refinement       a fixed number of 3x3 block-Jacobi PCG iterations on
//                    H_lag d_f = -g - H d_s from d_f = 0 (Sec. 3.8.2), where
//                    H_lag holds the elastic and inertia part of H from the
//                    last refresh plus the current barrier curvature;
//   line search      CCD filter and Armijo backtracking on d = d_s + d_f.
// The lagged part is refreshed at the first iteration and whenever the mean
// of the last lag_window accepted step sizes falls below lag_threshold, at
// most once every lag_min_gap iterations.  The iteration stops once the
// mean per-vertex norm of d_s divided by h is below paper_eps (m/s).
// U_a is the per-object affine basis restricted by the weights
// phi_a(v) = sum_i phi_i(v) (= 1 - phi_DBC(v) with Dirichlet vertices).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <deque>
#include <numeric>
#include <vector>

#include "ms_internal.h"
#include "reduce.h"

namespace ms {

namespace {

struct Aff {
  double o[3];
};

__device__ __forceinline__ double aff_p(const double* rest, int64_t v, Aff a, int l) {
  return l == 0 ? 1.0 : rest[3 * v + l - 1] - a.o[l - 1];
}

// out_v = phi_a(v) p_l(v) e_comp, the lifted k-th affine basis vector
// (k = 4 comp + l), zero on pinned vertices.
__global__ void k_affine_lift(int64_t n, const double* __restrict__ phia, const double* __restrict__ rest, Aff a,
                              int k, double* __restrict__ out) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int comp = k / 4, l = k % 4;
  const double val = phia[v] * aff_p(rest, v, a, l);
#pragma unroll
  for (int i = 0; i < 3; ++i) out[3 * v + i] = i == comp ? val : 0.0;
}

// out[12] = U_a^T y (fixed-order grid reduction); pinned rows of y ignored.
__global__ void __launch_bounds__(256) k_affine_restrict(int64_t n, const double* __restrict__ phia,
                                                         const double* __restrict__ rest, Aff a,
                                                         const double* __restrict__ y,
                                                         const uint8_t* __restrict__ pinned,
                                                         double* __restrict__ part, unsigned* __restrict__ counter,
                                                         double* __restrict__ out) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double acc[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) acc[q] = 0.0;
  if (v < n && !pinned[v]) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const double w = phia[v] * aff_p(rest, v, a, l);
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) acc[4 * comp + l] = w * y[3 * v + comp];
    }
  }
  if (grid_sum<12>(acc, part, counter) && threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 12; ++q) out[q] = acc[q];
}

// d_v = phi_a(v) (t + A (x_v - o)) with q = [t_0, A_0., t_1, A_1., t_2, A_2.].
__global__ void k_affine_apply(int64_t n, const double* __restrict__ phia, const double* __restrict__ rest, Aff a,
                               const double* __restrict__ q, double* __restrict__ d) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l) s += q[4 * comp + l] * aff_p(rest, v, a, l);
    d[3 * v + comp] = phia[v] * s;
  }
}

// out = pinned ? 0 : a g + b t, componentwise.
__global__ void k_combine(int64_t n, double a, const double* __restrict__ g, double b, const double* __restrict__ t,
                          const uint8_t* __restrict__ pinned, double* __restrict__ out) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
#pragma unroll
  for (int i = 0; i < 3; ++i) out[3 * v + i] = pinned[v] ? 0.0 : a * g[3 * v + i] + b * t[3 * v + i];
}

// out[0] = sum_v ||d_v||.
__global__ void __launch_bounds__(256) k_vnorm_sum(int64_t n, const double* __restrict__ d,
                                                   double* __restrict__ part, unsigned* __restrict__ counter,
                                                   double* __restrict__ out) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double acc[1] = {0.0};
  if (v < n) acc[0] = sqrt(d[3 * v] * d[3 * v] + d[3 * v + 1] * d[3 * v + 1] + d[3 * v + 2] * d[3 * v + 2]);
  if (grid_sum<1>(acc, part, counter) && threadIdx.x == 0) out[0] = acc[0];
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

unsigned nb(int64_t n) { return unsigned((n + 255) / 256); }

// Exact solve of the symmetric 12x12 affine system (Cholesky; a pivot below
// 1e-14 of the largest diagonal entry is replaced by that entry, which
// leaves directions the weights cannot move at zero).
void solve12(const double* A, const double* b, double* q) {
  double L[12][12] = {};
  double dmax = 0.0;
  for (int i = 0; i < 12; ++i) dmax = std::max(dmax, A[13 * i]);
  if (!(dmax > 0.0)) dmax = 1.0;
  for (int j = 0; j < 12; ++j) {
    double d = 0.5 * (A[12 * j + j] + A[12 * j + j]);
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 1e-14 * dmax)) d = dmax;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 12; ++i) {
      double s = 0.5 * (A[12 * i + j] + A[12 * j + i]);
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      L[i][j] = s / L[j][j];
    }
  }
  double y[12];
  for (int i = 0; i < 12; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
    y[i] = s / L[i][i];
  }
  for (int i = 11; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 12; ++k) s -= L[k][i] * q[k];
    q[i] = s / L[i][i];
  }
}

ms_status ensure_paper_buffers(ms_ctx* c, int prec) {
  const int64_t n = c->n, slots9 = 9 * int64_t(c->pat.nslots);
  ms_status s;
  if (!c->d_ds) {
    if ((s = alloc_n(c, &c->d_ds, 3 * n)) || (s = alloc_n(c, &c->d_gsave, 3 * n)) ||
        (s = alloc_n(c, &c->d_aff, 12 * 12 + 24)))
      return s;
  }
  if (c->lag_prec != prec) {
    if (c->d_lag) dfree(c, c->d_lag);
    if (c->d_hlag) dfree(c, c->d_hlag);
    if (c->d_Dinv_lag) dfree(c, c->d_Dinv_lag);
    c->d_lag = c->d_hlag = c->d_Dinv_lag = nullptr;
    if (prec == MS_PREC_FP64) {
      double *a = nullptr, *b = nullptr, *d = nullptr;
      if ((s = alloc_n(c, &a, slots9)) || (s = alloc_n(c, &b, slots9)) || (s = alloc_n(c, &d, 9 * n))) return s;
      c->d_lag = a, c->d_hlag = b, c->d_Dinv_lag = d;
    } else {
      float *a = nullptr, *b = nullptr, *d = nullptr;
      if ((s = alloc_n(c, &a, slots9)) || (s = alloc_n(c, &b, slots9)) || (s = alloc_n(c, &d, 9 * n))) return s;
      c->d_lag = a, c->d_hlag = b, c->d_Dinv_lag = d;
    }
    c->lag_prec = prec;
  }
  return MS_OK;
}

// Swaps the Hessian values and block-Jacobi inverses of precision prec with
// the lagged ones for the duration of the refinement solve.
struct LagSwap {
  ms_ctx* c;
  int prec;
  bool graphs;
  LagSwap(ms_ctx* cc, int p) : c(cc), prec(p), graphs(cc->use_graphs) {
    swap();
    c->use_graphs = false;  // captured graphs hold the regular value pointers
  }
  ~LagSwap() {
    swap();
    c->use_graphs = graphs;
  }
  template <typename T>
  static void exchange(T*& a, void*& b) {
    T* t = a;
    a = static_cast<T*>(b);
    b = t;
  }
  void swap() {
    if (prec == MS_PREC_FP64) {
      exchange(c->d_vals, c->d_hlag);
      exchange(c->d_Dinv, c->d_Dinv_lag);
    } else {
      exchange(c->d_vals32, c->d_hlag);
      exchange(c->d_Dinv32, c->d_Dinv_lag);
    }
  }
};

}  // namespace

ms_status paper_step(ms_ctx* c, double dt, const ms_solver_params& P, ms_step_stats* st) {
  const double t0 = now_ms();
  if (!c->has_basis) return fail(c, MS_E_ORDER, "paper mode needs a basis");
  if (c->has_hs && c->hs_mu > 0.0) return fail(c, MS_E_ARG, "paper mode does not support friction");
  set_coarse_f32(c, false);
  c->has_prev = false;  // no BDF2 history across paper-mode steps
  const double h2 = dt * dt;
  const int prec = P.precision == MS_PREC_MIXED ? MS_PREC_MIXED : MS_PREC_FP64;
  ms_status s;
  if ((s = ensure_paper_buffers(c, prec))) return s;
  const int64_t n = c->n, n3 = 3 * n;
  const size_t vsz = prec == MS_PREC_FP64 ? sizeof(double) : sizeof(float);
  const size_t vbytes = vsz * 9 * size_t(c->pat.nslots);
  void* vals = prec == MS_PREC_FP64 ? static_cast<void*>(c->d_vals) : static_cast<void*>(c->d_vals32);
  const int refine = P.refine_iters > 0 ? P.refine_iters : c->refine_auto;
  Aff a;
  for (int i = 0; i < 3; ++i) a.o[i] = c->oa[i];
  launch_predict(c, dt);
  launch_apply_dbc(c, int64_t(c->h_dbc.size()));
  c->timing = false;
  ms_step_stats S{};
  S.min_alpha = 1.0;
  std::deque<double> alphas;
  int last_refresh = -1000000;
  bool converged = false;
  double dnorm = 0.0;
  int it = 0;
  for (; it < P.max_newton; ++it) {
    // g, H (PSD-projected), its Galerkin matrix and inverse
    if ((s = assemble(c, c->d_x, h2, prec, true, true, MS_PC_TWO_LEVEL_ADDITIVE, true))) break;
    // lagged elastic + inertia part, refreshed on the trigger
    bool refresh = it == 0;
    if (!refresh && int(alphas.size()) >= std::max(1, P.lag_window) && it - last_refresh >= P.lag_min_gap) {
      double avg = 0.0;
      for (int k = 0; k < P.lag_window; ++k) avg += alphas[alphas.size() - 1 - k];
      refresh = avg / P.lag_window < P.lag_threshold;
    }
    if (refresh) {
      MS_HIP(hipMemcpyAsync(c->d_lag, vals, vbytes, hipMemcpyDeviceToDevice, c->stream));
      launch_diag_barrier(c, prec, c->d_lag, c->d_x, h2, -1.0);
      last_refresh = it;
      ++S.hessian_refreshes;
    }
    MS_HIP(hipMemcpyAsync(c->d_hlag, c->d_lag, vbytes, hipMemcpyDeviceToDevice, c->stream));
    launch_diag_barrier(c, prec, c->d_hlag, c->d_x, h2, 1.0);
    // affine level: columns U_a^T H U_a e_k and U_a^T g
    for (int k = 0; k < 12; ++k) {
      k_affine_lift<<<nb(n), 256, 0, c->stream>>>(n, c->d_phia, c->d_rest, a, k, c->d_p);
      launch_spmv(c, prec, c->d_p, c->d_w);
      k_affine_restrict<<<nb(n), 256, 0, c->stream>>>(n, c->d_phia, c->d_rest, a, c->d_w, c->d_pinned, c->d_part,
                                                       c->d_counter, c->d_aff + 12 * k);
    }
    k_affine_restrict<<<nb(n), 256, 0, c->stream>>>(n, c->d_phia, c->d_rest, a, c->d_g, c->d_pinned, c->d_part,
                                                     c->d_counter, c->d_aff + 144);
    double haff[156], q[12], rhs[12];
    MS_HIP(hipMemcpyAsync(haff, c->d_aff, sizeof(haff), hipMemcpyDeviceToHost, c->stream));
    if ((s = sync(c))) break;
    for (int i = 0; i < 12; ++i) rhs[i] = -haff[144 + i];
    bool finite = true;
    for (double v : haff) finite = finite && std::isfinite(v);
    if (!finite) {
      s = fail(c, MS_E_NONFINITE, "non-finite affine system");
      break;
    }
    // haff holds columns: A[i][k] = haff[12 k + i]; solve12 reads row-major
    double Ar[144];
    for (int i = 0; i < 12; ++i)
      for (int k = 0; k < 12; ++k) Ar[12 * i + k] = haff[12 * k + i];
    solve12(Ar, rhs, q);
    MS_HIP(hipMemcpyAsync(c->d_aff + 156, q, sizeof(q), hipMemcpyHostToDevice, c->stream));
    k_affine_apply<<<nb(n), 256, 0, c->stream>>>(n, c->d_phia, c->d_rest, a, c->d_aff + 156, c->d_ds);
    // subspace level on r = -g - H d_s
    launch_spmv(c, prec, c->d_ds, c->d_w);
    k_combine<<<nb(n), 256, 0, c->stream>>>(n, -1.0, c->d_g, -1.0, c->d_w, c->d_pinned, c->d_r);
    launch_restrict(c, c->d_r, nullptr, nullptr);
    launch_coarse_gemv(c, prec, nullptr);
    launch_prolong_add(c, c->d_ds, nullptr);
    // termination measure of this iteration's subspace direction
    k_vnorm_sum<<<nb(n), 256, 0, c->stream>>>(n, c->d_ds, c->d_part, c->d_counter, c->d_scal + S_DOT2);
    // refinement: H_lag d_f = -g - H d_s, i.e. PCG on the gradient g + H d_s
    launch_spmv(c, prec, c->d_ds, c->d_w);
    MS_HIP(hipMemcpyAsync(c->d_gsave, c->d_g, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    k_combine<<<nb(n), 256, 0, c->stream>>>(n, 1.0, c->d_gsave, 1.0, c->d_w, c->d_pinned, c->d_g);
    int iters = 0, code = 0;
    {
      LagSwap swap(c, prec);
      launch_block_jacobi(c, prec);
      s = pcg_solve(c, prec, MS_PC_BLOCK_JACOBI, 1e-300, 1e-300, true, refine, &iters, &code, 0);
    }
    MS_HIP(hipMemcpyAsync(c->d_g, c->d_gsave, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (s) break;
    S.pcg_iters += iters;
    S.max_pcg_iters = std::max(S.max_pcg_iters, iters);
    const double ds_mean = c->h_scal[S_DOT2] / double(n);
    // d = d_f + d_s; fall back to d_s alone if the sum is not a descent direction
    launch_axpy(c, c->d_d, c->d_ds, 1.0, n3);
    launch_dots(c, c->d_g, c->d_d, c->d_d, c->d_d, nullptr, nullptr);
    if ((s = read_scal(c))) break;
    double gd = c->h_scal[S_DOT0];
    dnorm = std::sqrt(c->h_scal[S_DOT1]);
    if (!(gd < 0.0)) {
      MS_HIP(hipMemcpyAsync(c->d_d, c->d_ds, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      launch_dots(c, c->d_g, c->d_d, c->d_d, c->d_d, nullptr, nullptr);
      if ((s = read_scal(c))) break;
      gd = c->h_scal[S_DOT0];
      dnorm = std::sqrt(c->h_scal[S_DOT1]);
    }
    if (!std::isfinite(gd)) {
      s = fail(c, MS_E_NONFINITE, "non-finite search direction");
      break;
    }
    double alpha = 0.0;
    int nbt = 0;
    if (gd < 0.0) {
      if ((s = line_search(c, h2, gd, P.max_backtracks, &alpha, &nbt))) break;
      launch_axpy(c, c->d_x, c->d_d, alpha, n3);
    }
    S.backtracks += nbt;
    S.min_alpha = std::min(S.min_alpha, alpha);
    alphas.push_back(alpha);
    if (c->verbose)
      std::fprintf(stderr, "[ms paper] it %d refresh %d pcg %d |d_s|/h %.3e |d| %.3e alpha %.3g bt %d\n", it,
                   int(refresh), iters, ds_mean / dt, dnorm, alpha, nbt);
    if (ds_mean / dt < P.paper_eps || gd >= 0.0) {
      converged = true;
      ++it;
      break;
    }
  }
  if (s) {
    (void)hipMemcpyAsync(c->d_x, c->d_xt, 3 * c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
    return s;
  }
  if (!converged) {
    (void)hipMemcpyAsync(c->d_x, c->d_xt, 3 * c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
    return fail(c, MS_E_NOCONV, "paper-mode Newton did not meet its termination rule");
  }
  launch_velocity(c, 1.0 / dt);
  double ef[4];
  if ((s = energy(c, c->d_x, nullptr, 0.0, h2, ef))) return s;
  launch_dots(c, nullptr, nullptr, nullptr, nullptr, c->d_x, c->d_xt);
  if ((s = read_scal(c))) return s;
  S.newton_iters = it;
  S.energy = ef[0] + ef[1] + ef[2] + ef[3];
  S.last_dnorm = dnorm;
  S.disp_norm = std::sqrt(c->h_scal[S_DOT2]);
  S.time_ms = now_ms() - t0;
  if (st) *st = S;
  return MS_OK;
}

}  // namespace ms
