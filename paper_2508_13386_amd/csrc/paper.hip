// The paper's three-level inexact Newton timestep (Alg. 1 with the linear
// solves of Alg. 2, Sec. 3.7).
//
// Per Newton iteration, with g and the PSD-projected Hessian H at x:
//   subspace matrix  A = U_s^T H U_s (r x r, FP64; exact Galerkin product or
//                    the cubature of Sec. 3.8), formed once per iteration;
//   affine level     (U_a^T H U_a) q_a = -U_a^T g by PCG with the 12 x 12
//                    block-Jacobi preconditioner to relative residual
//                    subspace_rtol (Sec. 3.7.1).  The affine basis lies in
//                    the span of the sparse one (partition of unity):
//                    U_a = U_s C with C mapping the affine coefficients to
//                    every handle's (the constant part gains the offset of
//                    the handle origin from the affine origin), so the
//                    12 x 12 system is C^T A C and its right-hand side
//                    C^T U_s^T (-g);
//   sparse level     (U_s^T H U_s) q_s = U_s^T r with r = -g - H U_a q_a,
//                    i.e. right-hand side U_s^T (-g) - A C q_a, by PCG with
//                    one 12 x 12 Jacobi block per handle to the same
//                    relative residual; d_s = U_s (C q_a + q_s);
//   refinement       a fixed number (20 or 40 from the partitions' hop
//                    diameters, Sec. 3.7.2) of Jacobi-preconditioned PCG
//                    iterations on H_lag d_f = -g - H d_s from d_f = 0, where
//                    H_lag holds the elastic and inertia part of H from the
//                    last refresh plus the current barrier curvature;
//   line search      CCD filter and Armijo backtracking on d = d_s + d_f
//                    (Sec. 3.9).
// The lagged part is refreshed at the first iteration and whenever the mean
// of the last lag_window accepted step sizes falls below lag_threshold, at
// most once every lag_min_gap iterations.  The iteration stops once the
// mean per-vertex norm of d_s divided by h is below paper_eps (m/s).
//
// The subspace PCG runs entirely on the device: a 12 x 12 block inverse per
// handle (LDL^T generalised inverse, a pivot not above 1e-10 of its diagonal
// entry counting as zero), then per iteration one wave-per-row GEMV with A
// and one single-block update kernel (dots, step, recursive residual, stop
// test ||r|| <= rtol ||r_0||, preconditioner, new direction) that raises a
// device flag; the host looks at the flag once per chunk of iterations.
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

constexpr int kDp = 1024;       // threads of the single-block PCG kernels
constexpr int kDpChunk = 8;     // subspace PCG iterations between flag reads
// dense PCG state: [0] r.z, [1] stop threshold rtol^2 ||r_0||^2, [2] done,
// [3] iterations, [4] iteration cap
enum { DP_RZ = 0, DP_TOL2, DP_DONE, DP_IT, DP_MAX, DP_COUNT = 8 };

__device__ __forceinline__ double block_sum1(double v) {
  double a[1] = {v};
  block_sum<1>(a);
  return a[0];
}

// Generalised inverse of every 12 x 12 diagonal block of the dense matrix A
// (leading dimension lda): LDL^T in natural order, a pivot not above 1e-10
// of the block's original diagonal entry counts as zero, then
// X = L^-T D^+ L^-1.  One 64-thread block per handle.
__global__ void __launch_bounds__(64) k_block_ldl_pinv(int lda, const double* __restrict__ A,
                                                       double* __restrict__ X) {
  __shared__ double B[12][12], L[12][12], Li[12][12], dp[12];
  const int h = blockIdx.x, t = threadIdx.x;
  for (int q = t; q < 144; q += 64) {
    const int i = q / 12, j = q % 12;
    B[i][j] = A[int64_t(12 * h + i) * lda + 12 * h + j];
    L[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  if (t == 0) {
    double d[12];
    for (int j = 0; j < 12; ++j) {
      double dj = B[j][j];
      for (int q = 0; q < j; ++q) dj -= L[j][q] * L[j][q] * d[q];
      if (!(dj > 1e-10 * B[j][j])) {
        d[j] = 0.0;
        continue;
      }
      d[j] = dj;
      for (int i = j + 1; i < 12; ++i) {
        double s = B[i][j];
        for (int q = 0; q < j; ++q) s -= L[i][q] * L[j][q] * d[q];
        L[i][j] = s / dj;
      }
    }
    for (int j = 0; j < 12; ++j) dp[j] = d[j] > 0.0 ? 1.0 / d[j] : 0.0;
  }
  __syncthreads();
  // columns of L^-1 by forward substitution (unit lower triangular)
  if (t < 12) {
    double y[12];
    for (int i = 0; i < 12; ++i) {
      double s = i == t ? 1.0 : 0.0;
      for (int q = 0; q < i; ++q) s -= L[i][q] * y[q];
      y[i] = s;
    }
    for (int i = 0; i < 12; ++i) Li[i][t] = y[i];
  }
  __syncthreads();
  for (int q = t; q < 144; q += 64) {
    const int a = q / 12, b = q % 12;
    double s = 0.0;
    for (int j = 0; j < 12; ++j) s += Li[j][a] * dp[j] * Li[j][b];
    X[144 * int64_t(h) + q] = s;
  }
}

// z = blockdiag(X) r for dim = 12 nb entries (each thread some rows).
__device__ __forceinline__ void apply_blocks(int dim, const double* __restrict__ X, const double* __restrict__ r,
                                             double* __restrict__ z) {
  for (int i = threadIdx.x; i < dim; i += blockDim.x) {
    const int h = i / 12, a = i % 12;
    const double* xr = X + 144 * int64_t(h) + 12 * a;
    const double* rr = r + 12 * h;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 12; ++b) s += xr[b] * rr[b];
    z[i] = s;
  }
}

// x = 0, r = b, z = M r, p = z; state: r.z, stop threshold, done flag.
__global__ void __launch_bounds__(kDp) k_dpcg_init(int dim, double rtol, int max_it, const double* __restrict__ b,
                                                   const double* __restrict__ X, double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ z,
                                                   double* __restrict__ p, double* __restrict__ st) {
  double bb = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) {
    const double v = b[i];
    x[i] = 0.0;
    r[i] = v;
    bb += v * v;
  }
  bb = block_sum1(bb);
  __syncthreads();
  apply_blocks(dim, X, r, z);
  __syncthreads();
  double rz = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) {
    p[i] = z[i];
    rz += r[i] * z[i];
  }
  rz = block_sum1(rz);
  if (threadIdx.x == 0) {
    st[DP_RZ] = rz;
    st[DP_TOL2] = rtol * rtol * bb;
    // a zero right-hand side, or no iteration allowed: nothing to do
    st[DP_DONE] = (bb == 0.0 || max_it <= 0) ? 1.0 : 0.0;
    st[DP_IT] = 0.0;
    st[DP_MAX] = double(max_it);
  }
}

// q = A p, one wave per row, skipped once the solve is done.
__global__ void __launch_bounds__(256) k_dpcg_gemv(int dim, int lda, const double* __restrict__ A,
                                                   const double* __restrict__ p, double* __restrict__ q,
                                                   const double* __restrict__ st) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (st[DP_DONE] != 0.0 || row >= dim) return;
  const double* a = A + int64_t(row) * lda;
  double s = 0.0;
  for (int j = lane; j < dim; j += 64) s += a[j] * p[j];
  s = wave_sum(s);
  if (lane == 0) q[row] = s;
}

// One PCG update after q = A p: alpha, x, r, the stop test on the recursive
// residual, z = M r, beta, p.  A single block, so every reduction has one
// fixed order.
__global__ void __launch_bounds__(kDp) k_dpcg_update(int dim, const double* __restrict__ X, double* __restrict__ x,
                                                     double* __restrict__ r, double* __restrict__ z,
                                                     double* __restrict__ p, const double* __restrict__ q,
                                                     double* __restrict__ st) {
  __shared__ int stop;
  if (st[DP_DONE] != 0.0) return;
  double pq = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) pq += p[i] * q[i];
  pq = block_sum1(pq);
  if (!(pq > 0.0)) {  // loss of positive curvature: keep x
    if (threadIdx.x == 0) st[DP_DONE] = 1.0;
    return;
  }
  const double alpha = st[DP_RZ] / pq;
  double rr = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    rr += ri * ri;
  }
  rr = block_sum1(rr);
  if (threadIdx.x == 0) {
    const double it = st[DP_IT] + 1.0;
    st[DP_IT] = it;
    stop = (rr <= st[DP_TOL2] || it >= st[DP_MAX]) ? 1 : 0;
    if (stop) st[DP_DONE] = 1.0;
  }
  __syncthreads();
  if (stop) return;
  apply_blocks(dim, X, r, z);
  __syncthreads();
  double rz = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) rz += r[i] * z[i];
  rz = block_sum1(rz);
  const double beta = rz / st[DP_RZ];
  for (int i = threadIdx.x; i < dim; i += blockDim.x) p[i] = z[i] + beta * p[i];
  __syncthreads();
  if (threadIdx.x == 0) st[DP_RZ] = rz;
}

// Dense right-hand side from the restriction partials: out_(12 i + q) =
// sum of handle i's chunk partials q, in chunk order.
__global__ void k_coarse_rhs(int r, const int2* __restrict__ hinfo, const double* __restrict__ part,
                             double* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= r) return;
  const int2 hi = hinfo[idx / 12];
  const int q = idx % 12;
  double s = 0.0;
  for (int k = 0; k < hi.y; ++k) s += part[12 * int64_t(hi.x + k) + q];
  out[idx] = s;
}

// Y = A C (r x 12): column 4c + l of C has a one at every handle's entry
// (c, l) and, for l > 0, the offset delta_(j, l - 1) = (o_j - o_a)_(l-1) at
// the handle's constant entry (c, 0).  One wave per row.
__global__ void __launch_bounds__(256) k_affine_y(int r, int m, const double* __restrict__ A,
                                                  const double* __restrict__ delta, double* __restrict__ Y) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= r) return;
  const double* a = A + int64_t(row) * r;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int j = lane; j < m; j += 64) {
    const double* aj = a + 12 * j;
    const double d0 = delta[3 * j], d1 = delta[3 * j + 1], d2 = delta[3 * j + 2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double a0 = aj[4 * c];
      acc[4 * c] += a0;
      acc[4 * c + 1] += aj[4 * c + 1] + d0 * a0;
      acc[4 * c + 2] += aj[4 * c + 2] + d1 * a0;
      acc[4 * c + 3] += aj[4 * c + 3] + d2 * a0;
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = wave_sum(acc[k]);
  if (lane < 12) {
    double v = acc[0];
#pragma unroll
    for (int k = 1; k < 12; ++k)
      if (lane == k) v = acc[k];
    Y[12 * int64_t(row) + lane] = v;
  }
}

// The affine system C^T Y (12 x 12) and right-hand side C^T b; one block.
__global__ void __launch_bounds__(256) k_affine_system(int m, const double* __restrict__ Y,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ delta, double* __restrict__ Aa,
                                                       double* __restrict__ ba) {
  const int t = threadIdx.x;
  if (t >= 156) return;
  const int i = t < 144 ? t / 12 : t - 144;  // row of C^T: (c, l) = (i / 4, i % 4)
  const int k = t < 144 ? t % 12 : 0;
  const int c = i / 4, l = i % 4;
  double s = 0.0;
  for (int j = 0; j < m; ++j) {
    const int64_t rl = 12 * int64_t(j) + 4 * c + l, r0 = 12 * int64_t(j) + 4 * c;
    const double dl = l > 0 ? delta[3 * j + l - 1] : 0.0;
    if (t < 144)
      s += Y[12 * rl + k] + (l > 0 ? dl * Y[12 * r0 + k] : 0.0);
    else
      s += b[rl] + (l > 0 ? dl * b[r0] : 0.0);
  }
  if (t < 144)
    Aa[t] = s;
  else
    ba[i] = s;
}

// b2 = b - Y q_a (the sparse level's right-hand side).
__global__ void k_sparse_rhs(int r, const double* __restrict__ b, const double* __restrict__ Y,
                             const double* __restrict__ qa, double* __restrict__ b2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r) return;
  double s = b[i];
#pragma unroll
  for (int k = 0; k < 12; ++k) s -= Y[12 * int64_t(i) + k] * qa[k];
  b2[i] = s;
}

// e = C q_a + q_s.
__global__ void k_coarse_dir(int r, const double* __restrict__ delta, const double* __restrict__ qa,
                             const double* __restrict__ qs, double* __restrict__ e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r) return;
  const int j = i / 12, c = (i % 12) / 4, l = i % 4;
  double v = qa[4 * c + l];
  if (l == 0) v += delta[3 * j] * qa[4 * c + 1] + delta[3 * j + 1] * qa[4 * c + 2] + delta[3 * j + 2] * qa[4 * c + 3];
  e[i] = v + qs[i];
}

// out = pinned ? 0 : a g + b t, componentwise.
__global__ void k_combine(int64_t n, double a, const double* __restrict__ g, double b, const double* __restrict__ t,
                          const uint8_t* __restrict__ pinned, double* __restrict__ out) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
#pragma unroll
  for (int i = 0; i < 3; ++i) out[3 * v + i] = pinned[v] ? 0.0 : a * g[3 * v + i] + b * (t ? t[3 * v + i] : 0.0);
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

// Diagonal (Jacobi) preconditioner of the lagged Hessian in the 3x3 layout
// the PCG applies: Dinv_v = diag(1 / H_vv,aa), zero at pinned vertices.
template <typename VT>
__global__ void k_jacobi_diag(int64_t n, int S, const int32_t* __restrict__ diag_slot, const VT* __restrict__ vals,
                              const uint8_t* __restrict__ pinned, VT* __restrict__ Dinv) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const VT* a = vals + vbase(diag_slot[v], S);
  const bool pin = pinned && pinned[v];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    double val = 0.0;
    if (!pin && q % 4 == 0) {
      const double d = double(a[S * q]);
      val = d > 0.0 ? 1.0 / d : 0.0;
    }
    Dinv[9 * v + q] = VT(val);
  }
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

unsigned nb(int64_t n) { return unsigned((n + 255) / 256); }

ms_status ensure_paper_buffers(ms_ctx* c, int prec) {
  const int64_t n = c->n, slots9 = 9 * int64_t(c->pat.nslots);
  const int r = c->r, m = c->basis.m;
  ms_status s;
  if (!c->d_ds) {
    if ((s = alloc_n(c, &c->d_ds, 3 * n)) || (s = alloc_n(c, &c->d_gsave, 3 * n))) return s;
  }
  if (c->paper_r != r) {
    // [bs r][b2 r][qs r][x r][rr r][z r][p r][q r][Y 12r][X 144m][Aa 144][ba 12][qa 12][Xa 144][delta 3m][st 8]
    const size_t len = size_t(8) * r + 12 * size_t(r) + 144 * size_t(m) + 144 + 12 + 12 + 144 + 3 * size_t(m) + 8;
    if ((s = alloc_n(c, &c->d_paper, len))) return s;
    c->paper_r = r;
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

// Views into the paper-mode workspace.
struct PaperWs {
  double *bs, *b2, *qs, *x, *r, *z, *p, *q, *Y, *X, *Aa, *ba, *qa, *Xa, *delta, *st;
  PaperWs(ms_ctx* c) {
    const int64_t r_ = c->r, m = c->basis.m;
    double* w = c->d_paper;
    bs = w, b2 = bs + r_, qs = b2 + r_, x = qs + r_, r = x + r_, z = r + r_, p = z + r_, q = p + r_;
    Y = q + r_, X = Y + 12 * r_, Aa = X + 144 * m, ba = Aa + 144, qa = ba + 12, Xa = qa + 12, delta = Xa + 144;
    st = delta + 3 * m;
  }
};

// PCG on the dense dim x dim matrix A (leading dimension lda, FP64) with the
// 12 x 12 block-Jacobi preconditioner whose generalised inverses are in X,
// from zero to relative residual rtol; the solution is left in ws.x.
ms_status dense_block_pcg(ms_ctx* c, const PaperWs& ws, const double* A, int lda, int dim, const double* b,
                          const double* X, double rtol, int max_it, int* iters) {
  k_dpcg_init<<<1, kDp, 0, c->stream>>>(dim, rtol, max_it, b, X, ws.x, ws.r, ws.z, ws.p, ws.st);
  double st[DP_COUNT];
  const unsigned gb = unsigned((dim + 3) / 4);
  while (true) {
    for (int k = 0; k < kDpChunk; ++k) {
      k_dpcg_gemv<<<gb, 256, 0, c->stream>>>(dim, lda, A, ws.p, ws.q, ws.st);
      k_dpcg_update<<<1, kDp, 0, c->stream>>>(dim, X, ws.x, ws.r, ws.z, ws.p, ws.q, ws.st);
    }
    MS_HIP(hipMemcpyAsync(st, ws.st, sizeof(st), hipMemcpyDeviceToHost, c->stream));
    ms_status s = sync(c);
    if (s) return s;
    if (st[DP_DONE] != 0.0) break;
  }
  *iters = int(st[DP_IT]);
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
  if (!(P.subspace_rtol >= 0.0) || !(P.subspace_rtol < 1.0)) return fail(c, MS_E_ARG, "subspace_rtol must lie in [0, 1)");
  set_coarse_f32(c, false);
  c->has_prev = false;  // no BDF2 history across paper-mode steps
  const double h2 = dt * dt;
  const int prec = P.precision == MS_PREC_MIXED ? MS_PREC_MIXED : MS_PREC_FP64;
  ms_status s;
  if ((s = ensure_paper_buffers(c, prec))) return s;
  const int64_t n = c->n, n3 = 3 * n;
  const int r = c->r, m = c->basis.m;
  const size_t vsz = prec == MS_PREC_FP64 ? sizeof(double) : sizeof(float);
  const size_t vbytes = vsz * 9 * size_t(c->pat.nslots);
  void* vals = prec == MS_PREC_FP64 ? static_cast<void*>(c->d_vals) : static_cast<void*>(c->d_vals32);
  const int refine = P.refine_iters > 0 ? P.refine_iters : c->refine_auto;
  const int sub_max = P.max_pcg > 0 ? P.max_pcg : 1;
  PaperWs ws(c);
  // handle-origin offsets from the affine origin (the entries of C)
  c->h_delta.resize(3 * size_t(m));
  for (int j = 0; j < m; ++j)
    for (int d = 0; d < 3; ++d) c->h_delta[3 * j + d] = c->basis.origins[3 * j + d] - c->oa[d];
  MS_HIP(hipMemcpyAsync(ws.delta, c->h_delta.data(), 3 * size_t(m) * sizeof(double), hipMemcpyHostToDevice,
                        c->stream));
  launch_predict(c, dt);
  launch_apply_dbc(c, int64_t(c->h_dbc.size()));
  c->timing = false;
  ms_step_stats S{};
  S.min_alpha = 1.0;
  S.refine_iters = refine;
  std::deque<double> alphas;
  int last_refresh = -1000000;
  bool converged = false;
  double dnorm = 0.0;
  int it = 0;
  for (; it < P.max_newton; ++it) {
    // g, H (PSD-projected) and the subspace matrix A
    if ((s = assemble(c, c->d_x, h2, prec, true, false, MS_PC_BLOCK_JACOBI, false))) break;
    if ((s = launch_galerkin(c, prec, c->d_x, h2))) break;
    c->coarse_valid = 0;  // A now differs from the matrix the inverse was formed from
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
    // b_s = U_s^T (-g)
    k_combine<<<nb(n), 256, 0, c->stream>>>(n, -1.0, c->d_g, 0.0, nullptr, c->d_pinned, c->d_r);
    launch_restrict(c, c->d_r, nullptr, nullptr);
    k_coarse_rhs<<<nb(r), 256, 0, c->stream>>>(r, c->basis.d_hinfo, c->basis.d_rpart, ws.bs);
    // affine level: C^T A C q_a = C^T b_s
    k_affine_y<<<unsigned((r + 3) / 4), 256, 0, c->stream>>>(r, m, c->d_Ac, ws.delta, ws.Y);
    k_affine_system<<<1, 256, 0, c->stream>>>(m, ws.Y, ws.bs, ws.delta, ws.Aa, ws.ba);
    k_block_ldl_pinv<<<1, 64, 0, c->stream>>>(12, ws.Aa, ws.Xa);
    int ia = 0, is = 0;
    if ((s = dense_block_pcg(c, ws, ws.Aa, 12, 12, ws.ba, ws.Xa, P.subspace_rtol, sub_max, &ia))) break;
    MS_HIP(hipMemcpyAsync(ws.qa, ws.x, 12 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    // sparse level: A q_s = b_s - A C q_a
    k_sparse_rhs<<<nb(r), 256, 0, c->stream>>>(r, ws.bs, ws.Y, ws.qa, ws.b2);
    k_block_ldl_pinv<<<unsigned(m), 64, 0, c->stream>>>(r, c->d_Ac, ws.X);
    if ((s = dense_block_pcg(c, ws, c->d_Ac, r, r, ws.b2, ws.X, P.subspace_rtol, sub_max, &is))) break;
    S.subspace_pcg_iters += ia + is;
    // d_s = U_s (C q_a + q_s)
    k_coarse_dir<<<nb(r), 256, 0, c->stream>>>(r, ws.delta, ws.qa, ws.x, c->d_e);
    launch_fill(c, c->d_ds, 0.0, n3);
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
      if (prec == MS_PREC_FP64)
        k_jacobi_diag<double><<<nb(n), 256, 0, c->stream>>>(n, c->pat.S, c->pat.d_diag_slot, c->d_vals, c->d_pinned,
                                                            c->d_Dinv);
      else
        k_jacobi_diag<float><<<nb(n), 256, 0, c->stream>>>(n, c->pat.S, c->pat.d_diag_slot, c->d_vals32, c->d_pinned,
                                                           c->d_Dinv32);
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
      std::fprintf(stderr, "[ms paper] it %d refresh %d sub %d+%d pcg %d |d_s|/h %.3e |d| %.3e alpha %.3g bt %d\n",
                   it, int(refresh), ia, is, iters, ds_mean / dt, dnorm, alpha, nbt);
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
  // energy and displacement before the velocity update, so that a failure
  // here leaves x and v as they were
  double ef[4];
  s = energy(c, c->d_x, nullptr, 0.0, h2, ef);
  if (!s) {
    launch_dots(c, nullptr, nullptr, nullptr, nullptr, c->d_x, c->d_xt);
    s = read_scal(c);
  }
  if (s) {
    (void)hipMemcpyAsync(c->d_x, c->d_xt, 3 * c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
    return s;
  }
  launch_velocity(c, 1.0 / dt);
  S.newton_iters = it;
  S.energy = ef[0] + ef[1] + ef[2] + ef[3];
  S.last_dnorm = dnorm;
  S.disp_norm = std::sqrt(c->h_scal[S_DOT2]);
  S.time_ms = now_ms() - t0;
  if (st) *st = S;
  return MS_OK;
}

}  // namespace ms
