// Sparse products and preconditioned conjugate gradient for H d = -g
// (the Newton system of Sec. 3.1), on the sliced BSR3 layout.
//
// PCG uses the Chronopoulos-Gear recurrence, which needs one grid-wide
// reduction per iteration: per iteration two kernels run,
//   k_cg_spmv    w = H u and per-block partials of (r.u, w.u, r.r);
//   k_cg_update  every block sums the partials in the same fixed order, forms
//                alpha, beta and the convergence test, then p = u + beta p,
//                s = w + beta s, d += alpha p, r -= alpha s, u = S r (3x3
//                block-Jacobi; the two-level preconditioner adds its coarse
//                correction in separate kernels).
// A wave serves one slice of S rows with 64/S lanes per row (S = 16, 32, 64),
// the lanes of a row striding over its block columns and combining their
// sums with cross-lane shuffles.
// Every kernel returns at once when the device "done" flag is set, so fixed
// chunks of iterations can be captured in a HIP graph and replayed with one
// host synchronisation per chunk.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include <hip/hip_ext.h>

#include "cg_device.h"
#include "ms_internal.h"
#include "reduce.h"

namespace ms {

// One slice per wave, 4 waves per block.
template <typename VT, typename XT, int S>
__global__ void __launch_bounds__(256) k_spmv(int64_t n, int64_t nslices, const int32_t* __restrict__ slice_base,
                                              const int32_t* __restrict__ scol, const VT* __restrict__ vals,
                                              const XT* __restrict__ x, XT* __restrict__ y,
                                              const uint8_t* __restrict__ pinned) {
  const int64_t s = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (s >= nslices) return;
  const int lane = threadIdx.x & 63;
  double acc[3];
  row_product<VT, XT, S>(s, lane, slice_base, scol, vals, x, acc);
  const int64_t row = s * S + lane % S;
  if (lane < S && row < n) {
    const bool pin = pinned && pinned[row];
    y[3 * row] = pin ? XT(0) : XT(acc[0]);
    y[3 * row + 1] = pin ? XT(0) : XT(acc[1]);
    y[3 * row + 2] = pin ? XT(0) : XT(acc[2]);
  }
}

// ---------------------------------------------------------------------------
// PCG kernels.  VT is the type of the Hessian values and of the block-Jacobi
// inverse (double, or float in mixed precision); every vector, product
// accumulation and dot product is FP64.
// ---------------------------------------------------------------------------
// Recurrence state of one PCG iteration, double-buffered between
// iterations: [gamma_old, alpha_old, iter].
// w = H u and the block partials of (r.u, w.u, r.r); no grid-wide step here:
// the update kernel reduces the partials.
template <typename VT, int S>
__global__ void __launch_bounds__(256) k_cg_spmv(int64_t n, int64_t nslices, const int32_t* __restrict__ slice_base,
                                                 const int32_t* __restrict__ scol, const VT* __restrict__ vals,
                                                 const double* __restrict__ u, double* __restrict__ w,
                                                 const double* __restrict__ r, const uint8_t* __restrict__ pinned,
                                                 const double* __restrict__ scal, double* __restrict__ part) {
  const double done = scal[S_DONE];
  const int64_t s = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t row = s * S + lane % S;
  const bool has = s < nslices;
  const int base = has ? slice_base[s] : 0;
  const int width = has ? (slice_base[s + 1] - base) / S : 0;
  if (done != 0.0) return;  // the flag is the same for the whole grid
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


// Every block reduces the SpMV partials in the same order (identical,
// deterministic scalars in all blocks), block 0 records the recurrence state
// and the done flag, then p = u + beta p, s = w + beta s, d += alpha p,
// r -= alpha s, u = S r.  The vector operands are loaded before the partials
// are reduced so that both memory latencies overlap.
template <typename VT>
__global__ void __launch_bounds__(kUpdBlock) k_cg_update(int64_t n, int nparts, const double* __restrict__ part,
                                                         const double* __restrict__ st_in, double* __restrict__ st_out,
                                                         double* __restrict__ p, double* __restrict__ s,
                                                         double* __restrict__ d, double* __restrict__ r,
                                                         double* __restrict__ u, const double* __restrict__ w,
                                                         const VT* __restrict__ Dinv, double* __restrict__ scal) {
  const double done = scal[S_DONE];
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
  if (done != 0.0) return;  // the flag is the same for the whole grid
  double dots[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < 3; ++i) dots[i] += part[3 * b + i];
  block_sum<3>(dots);
  double alpha, beta;
  const int code = cg_scalars(st_in, scal, dots[0], dots[1], dots[2], alpha, beta);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
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


// d = 0, r = -g (zero on pinned DOFs), u = S r, p = s = 0; rho0 = r.r and the
// PCG scalars are initialised in the last block, with the forcing term
// eta = clamp(sqrt(||g|| / ||g_first||), eta_min, eta_max) of this Newton
// iteration.
template <typename VT>
__global__ void __launch_bounds__(256) k_cg_init(int64_t n, const double* __restrict__ g,
                                                 const uint8_t* __restrict__ pinned, double* __restrict__ p,
                                                 double* __restrict__ s, double* __restrict__ d, double* __restrict__ r,
                                                 double* __restrict__ u, const VT* __restrict__ Dinv, double eta_max,
                                                 double eta_min, int first, int forcing, double maxit,
                                                 double* __restrict__ st0, double* __restrict__ scal,
                                                 double* __restrict__ part,
                                                 unsigned* __restrict__ counter) {
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
  if (grid_sum<1>(rho, part, counter) && threadIdx.x == 0) {
    scal[S_RHO0] = rho[0];
    scal[S_RHO] = rho[0];
    if (first) scal[S_G0SQ] = rho[0];
    double eta;
    if (forcing == 1) {
      // Eisenstat-Walker choice 2 (gamma 0.9, exponent 2) with its safeguard
      if (first || !(scal[S_GPREV] > 0.0)) {
        eta = eta_max;
      } else {
        eta = 0.9 * rho[0] / scal[S_GPREV];  // 0.9 (||g_k|| / ||g_k-1||)^2
        const double safe = 0.9 * scal[S_ETAPREV] * scal[S_ETAPREV];
        if (safe > 0.1) eta = fmax(eta, safe);
      }
    } else {
      eta = scal[S_G0SQ] > 0.0 ? sqrt(sqrt(rho[0] / scal[S_G0SQ])) : 1.0;
    }
    eta = fmin(eta_max, fmax(eta_min, eta));
    scal[S_GPREV] = rho[0];
    scal[S_ETAPREV] = eta;
    scal[S_ETA] = eta;
    scal[S_TOL2] = eta * eta * rho[0];
    scal[S_ITER] = 0.0;
    scal[S_MAXIT] = maxit;
    st0[ST_GAMMA] = 0.0;
    st0[ST_ALPHA] = 1.0;
    st0[ST_ITER] = 0.0;
    scal[S_DONE] = rho[0] > 0.0 ? 0.0 : 1.0;
  }
}

// Inverse of each diagonal 3x3 block (cofactor formula in double); pinned
// vertices get a zero block so that the preconditioned vectors vanish there.
template <typename VT>
__global__ void k_block_jacobi(int64_t n, int S, const int32_t* __restrict__ diag_slot,
                               const VT* __restrict__ vals, const uint8_t* __restrict__ pinned,
                               VT* __restrict__ Dinv) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t slot = diag_slot[v];
  const VT* a = vals + vbase(slot, S);
  double m[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) m[c] = double(a[S * c]);
  double inv[9];
  inv[0] = m[4] * m[8] - m[5] * m[7];
  inv[1] = m[2] * m[7] - m[1] * m[8];
  inv[2] = m[1] * m[5] - m[2] * m[4];
  inv[3] = m[5] * m[6] - m[3] * m[8];
  inv[4] = m[0] * m[8] - m[2] * m[6];
  inv[5] = m[2] * m[3] - m[0] * m[5];
  inv[6] = m[3] * m[7] - m[4] * m[6];
  inv[7] = m[1] * m[6] - m[0] * m[7];
  inv[8] = m[0] * m[4] - m[1] * m[3];
  const double det = m[0] * inv[0] + m[1] * inv[3] + m[2] * inv[6];
  const double id = (pinned && pinned[v]) ? 0.0 : 1.0 / det;
#pragma unroll
  for (int c = 0; c < 9; ++c) Dinv[9 * v + c] = VT(inv[c] * id);
}

// Up to three masked dot products (null pairs skipped); the optional
// "minus" vectors give (a - am).(b - bm).
__global__ void __launch_bounds__(256) k_dots(int64_t len, const double* __restrict__ a0,
                                              const double* __restrict__ b0, const double* __restrict__ a1,
                                              const double* __restrict__ b1, const double* __restrict__ a2,
                                              const double* __restrict__ am2, double* __restrict__ part,
                                              unsigned* __restrict__ counter, double* __restrict__ out) {
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
  if (grid_sum<3>(v, part, counter) && threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = v[k];
}

__global__ void k_axpy(int64_t len, double* __restrict__ y, const double* __restrict__ x, double alpha) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < len) y[i] += alpha * x[i];
}
__global__ void k_fill(int64_t len, double* __restrict__ y, double v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < len) y[i] = v;
}
template <typename VT>
__global__ void k_extract(int64_t nnzb, int S, const int64_t* __restrict__ slot_of, const VT* __restrict__ vals,
                          double* __restrict__ out) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  const int64_t slot = slot_of[b];
  const VT* a = vals + vbase(slot, S);
#pragma unroll
  for (int c = 0; c < 9; ++c) out[9 * b + c] = double(a[S * c]);
}

// t = r - H x (zero on pinned rows); x is the iteration vector (VT) or the
// FP64 solution d.  In-place use (t == r) is safe: each row reads only its
// own r entry.
template <typename VT, int S>
__global__ void __launch_bounds__(256) k_spmv_resid(int64_t n, int64_t nslices, const int32_t* __restrict__ slice_base,
                                                    const int32_t* __restrict__ scol, const VT* __restrict__ vals,
                                                    const double* __restrict__ x, const double* r, double* t,
                                                    const uint8_t* __restrict__ pinned,
                                                    const double* __restrict__ scal) {
  if (scal[S_DONE] != 0.0) return;
  const int64_t s = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (s >= nslices) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = s * S + lane % S;
  double acc[3];
  row_product<VT, double, S>(s, lane, slice_base, scol, vals, x, acc);
  if (lane < S && row < n) {
    const bool pin = pinned[row];
#pragma unroll
    for (int i = 0; i < 3; ++i) t[3 * row + i] = pin ? 0.0 : r[3 * row + i] - acc[i];
  }
}

template <typename VT>
__global__ void __launch_bounds__(256) k_bj(int64_t n, const double* __restrict__ r, double* __restrict__ u,
                                            const VT* __restrict__ Dinv, const double* __restrict__ scal) {
  if (scal[S_DONE] != 0.0) return;
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double rr[3] = {r[3 * v], r[3 * v + 1], r[3 * v + 2]}, uu[3];
  bj_apply<VT>(Dinv, v, rr, uu);
#pragma unroll
  for (int i = 0; i < 3; ++i) u[3 * v + i] = uu[i];
}

static inline unsigned nblocks(int64_t n, int b) { return unsigned((n + b - 1) / b); }


void launch_spmv_resid(ms_ctx* c, int prec, bool from_d) {
  const int64_t ns = c->pat.nslices;
  const unsigned nbs = unsigned((ns + 3) / 4);
  const double* x = from_d ? c->d_d : c->d_u;
  double* t = from_d ? c->d_r : c->d_w;
  with_slice(c->pat.S, [&](auto SS) {
    constexpr int S = decltype(SS)::value;
    if (prec == MS_PREC_FP64)
      k_spmv_resid<double, S><<<nbs, 256, 0, c->stream>>>(c->n, ns, c->pat.d_slice_base, c->pat.d_col, c->d_vals, x,
                                                          c->d_r, t, c->d_pinned, c->d_scal);
    else
      k_spmv_resid<float, S><<<nbs, 256, 0, c->stream>>>(c->n, ns, c->pat.d_slice_base, c->pat.d_col, c->d_vals32, x,
                                                         c->d_r, t, c->d_pinned, c->d_scal);
  });
}

void launch_bj(ms_ctx* c, int prec) {
  if (prec == MS_PREC_FP64)
    k_bj<double><<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, c->d_r, c->d_u, c->d_Dinv, c->d_scal);
  else
    k_bj<float><<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, c->d_r, c->d_u, c->d_Dinv32, c->d_scal);
}

void launch_spmv(ms_ctx* c, int prec, const double* x, double* y) {
  const int64_t ns = c->pat.nslices;
  with_slice(c->pat.S, [&](auto SS) {
    constexpr int S = decltype(SS)::value;
    if (prec == MS_PREC_FP64)
      k_spmv<double, double, S><<<unsigned((ns + 3) / 4), 256, 0, c->stream>>>(c->n, ns, c->pat.d_slice_base,
                                                                               c->pat.d_col, c->d_vals, x, y, nullptr);
    else
      k_spmv<float, double, S><<<unsigned((ns + 3) / 4), 256, 0, c->stream>>>(c->n, ns, c->pat.d_slice_base,
                                                                              c->pat.d_col, c->d_vals32, x, y, nullptr);
  });
}

// Average duration (ms) of an FP64 SpMV on a candidate layout with random
// values; -1 on a HIP error.
double time_spmv_layout(ms_ctx* c, int S, const int32_t* d_slice_base, const int32_t* d_col, int64_t nslices,
                        int64_t nslots, int reps) {
  double *vals = nullptr, *x = nullptr, *y = nullptr;
  if (alloc_n(c, &vals, 9 * nslots) || alloc_n(c, &x, 3 * c->n) || alloc_n(c, &y, 3 * c->n)) return -1.0;
  k_fill<<<nblocks(9 * nslots, 256), 256, 0, c->stream>>>(9 * nslots, vals, 0.5);
  k_fill<<<nblocks(3 * c->n, 256), 256, 0, c->stream>>>(3 * c->n, x, 1.0);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
  auto run = [&]() {
    with_slice(S, [&](auto SS) {
      constexpr int SV = decltype(SS)::value;
      k_spmv<double, double, SV><<<unsigned((nslices + 3) / 4), 256, 0, c->stream>>>(c->n, nslices, d_slice_base,
                                                                                     d_col, vals, x, y, nullptr);
    });
  };
  for (int i = 0; i < 3; ++i) run();
  (void)hipEventRecord(e0, c->stream);
  for (int i = 0; i < reps; ++i) run();
  (void)hipEventRecord(e1, c->stream);
  float ms = -1.0f;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = -1.0f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dfree(c, vals);
  dfree(c, x);
  dfree(c, y);
  return ms < 0 ? -1.0 : double(ms) / reps;
}

void launch_block_jacobi(ms_ctx* c, int prec) {
  if (prec == MS_PREC_FP64)
    k_block_jacobi<double><<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, c->pat.S, c->pat.d_diag_slot, c->d_vals,
                                                                     c->d_pinned, c->d_Dinv);
  else
    k_block_jacobi<float><<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, c->pat.S, c->pat.d_diag_slot,
                                                                    c->d_vals32, c->d_pinned, c->d_Dinv32);
}

void launch_dots(ms_ctx* c, const double* a0, const double* b0, const double* a1, const double* b1,
                 const double* a2, const double* am2) {
  const int64_t len = 3 * c->n;
  k_dots<<<nblocks(len, 256), 256, 0, c->stream>>>(len, a0, b0, a1, b1, a2, am2, c->d_part, c->d_counter,
                                                   c->d_scal + S_DOT0);
}
void launch_axpy(ms_ctx* c, double* y, const double* x, double alpha, int64_t len) {
  k_axpy<<<nblocks(len, 256), 256, 0, c->stream>>>(len, y, x, alpha);
}
void launch_fill(ms_ctx* c, double* p, double v, int64_t len) {
  k_fill<<<nblocks(len, 256), 256, 0, c->stream>>>(len, p, v);
}
void launch_extract_bsr(ms_ctx* c, const int64_t* slot_of, int64_t nnzb, double* out, int prec) {
  if (prec == MS_PREC_FP64)
    k_extract<double><<<nblocks(nnzb, 256), 256, 0, c->stream>>>(nnzb, c->pat.S, slot_of, c->d_vals, out);
  else
    k_extract<float><<<nblocks(nnzb, 256), 256, 0, c->stream>>>(nnzb, c->pat.S, slot_of, c->d_vals32, out);
}

void launch_cg_init(ms_ctx* c, int prec, double eta_max, double eta_min, bool first, int max_it, int forcing) {
  const unsigned nb = nblocks(c->n, 256);
  if (prec == MS_PREC_FP64)
    k_cg_init<double><<<nb, 256, 0, c->stream>>>(c->n, c->d_g, c->d_pinned, c->d_p, c->d_s, c->d_d, c->d_r, c->d_u,
                                                 c->d_Dinv, eta_max, eta_min, first ? 1 : 0, forcing, double(max_it), c->d_cgst, c->d_scal, c->d_part,
                                                 c->d_counter);
  else
    k_cg_init<float><<<nb, 256, 0, c->stream>>>(c->n, c->d_g, c->d_pinned, c->d_p, c->d_s, c->d_d, c->d_r, c->d_u,
                                                c->d_Dinv32, eta_max, eta_min, first ? 1 : 0, forcing, double(max_it), c->d_cgst, c->d_scal, c->d_part,
                                                c->d_counter);
}

// One PCG iteration; `parity` selects the recurrence-state buffers
// (iteration k reads state k % 2 and writes (k + 1) % 2).
void launch_cg_update(ms_ctx* c, int prec, int parity) {
  const unsigned nbs = unsigned((c->pat.nslices + 3) / 4), nb = nblocks(c->n, kUpdBlock);
  const double* st_in = c->d_cgst + ST_N * parity;
  double* st_out = c->d_cgst + ST_N * (1 - parity);
  if (prec == MS_PREC_FP64)
    k_cg_update<double><<<nb, kUpdBlock, 0, c->stream>>>(c->n, int(nbs), c->d_part, st_in, st_out, c->d_p, c->d_s,
                                                         c->d_d, c->d_r, c->d_u, c->d_w, c->d_Dinv, c->d_scal);
  else
    k_cg_update<float><<<nb, kUpdBlock, 0, c->stream>>>(c->n, int(nbs), c->d_part, st_in, st_out, c->d_p, c->d_s,
                                                        c->d_d, c->d_r, c->d_u, c->d_w, c->d_Dinv32, c->d_scal);
}

// Average duration of `reps` back-to-back launches of one kernel of the PCG
// loop on the current buffers (1 update, 2 restriction, 3 coarse GEMV,
// 4 prolongation, 5 one whole iteration), with its algorithmic bytes.
ms_status time_loop_kernel(ms_ctx* c, int kernel, int prec, int reps, double* avg_us, double* bytes) {
  const int pc = c->has_basis ? MS_PC_TWO_LEVEL_ADDITIVE : MS_PC_BLOCK_JACOBI;
  if (kernel >= 2 && kernel <= 4 && !c->has_basis) return fail(c, MS_E_ORDER, "no basis");
  const double n = double(c->n), vb = prec == MS_PREC_FP64 ? 8.0 : 4.0;
  const double nnz = double(c->basis.nnz), r = double(c->r);
  auto run = [&]() {
    switch (kernel) {
      case 1: launch_cg_update(c, prec, 0); break;
      case 2: launch_restrict(c, c->d_r, nullptr, c->d_scal); break;
      case 3: launch_coarse_gemv(c, prec, c->d_scal); break;
      case 4: launch_prolong_add(c, c->d_u, c->d_scal); break;
      default: launch_cg_iteration(c, prec, pc, 0); break;
    }
  };
  switch (kernel) {
    case 1: *bytes = n * (6 * 24 + 9 * vb) + n * 5 * 24; break;
    case 2: *bytes = nnz * (4 + 32) + 24 * n + 8 * r; break;
    case 3: *bytes = r * r * (prec == MS_PREC_FP64 ? 8 : 4) + 16 * r; break;
    case 4: *bytes = 4 * n + nnz * (4 + 32) + 8 * r + 48 * n + n; break;
    default: *bytes = 0.0; break;
  }
  MS_HIP(hipMemsetAsync(c->d_scal + S_DONE, 0, sizeof(double), c->stream));
  for (int i = 0; i < 3; ++i) run();
  hipEvent_t e0, e1;
  MS_HIP(hipEventCreate(&e0));
  MS_HIP(hipEventCreate(&e1));
  MS_HIP(hipEventRecord(e0, c->stream));
  for (int i = 0; i < reps; ++i) {
    // the update may flag convergence, which would turn later replays into
    // early exits; it and the whole iteration re-clear the flag (a memset
    // between launches, included in their time)
    if (kernel == 1 || kernel == 5) MS_HIP(hipMemsetAsync(c->d_scal + S_DONE, 0, sizeof(double), c->stream));
    run();
  }
  MS_HIP(hipEventRecord(e1, c->stream));
  MS_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  MS_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_us = 1e3 * double(ms) / reps;
  return MS_OK;
}

void launch_cg_iteration(ms_ctx* c, int prec, int pc, int parity, hipEvent_t ev0, hipEvent_t ev1) {
  const int64_t ns = c->pat.nslices;
  const unsigned nbs = unsigned((ns + 3) / 4), nb = nblocks(c->n, kUpdBlock);
  const double* st_in = c->d_cgst + ST_N * parity;
  double* st_out = c->d_cgst + ST_N * (1 - parity);
  with_slice(c->pat.S, [&](auto SS) {
    constexpr int S = decltype(SS)::value;
    auto go = [&](auto kernel, const auto* vals) {
      if (ev0)  // the events take the dispatch's own start and end timestamps
        hipExtLaunchKernelGGL(kernel, dim3(nbs), dim3(256), 0, c->stream, ev0, ev1, 0, c->n, ns,
                              (const int32_t*)c->pat.d_slice_base, (const int32_t*)c->pat.d_col, vals,
                              (const double*)c->d_u, c->d_w, (const double*)c->d_r, (const uint8_t*)c->d_pinned,
                              (const double*)c->d_scal, c->d_part);
      else
        kernel<<<nbs, 256, 0, c->stream>>>(c->n, ns, c->pat.d_slice_base, c->pat.d_col, vals, c->d_u, c->d_w, c->d_r,
                                           c->d_pinned, c->d_scal, c->d_part);
    };
    if (prec == MS_PREC_FP64)
      go(k_cg_spmv<double, S>, (const double*)c->d_vals);
    else
      go(k_cg_spmv<float, S>, (const float*)c->d_vals32);
  });
  if (c->smoother)
    launch_cg_update_agg(c, prec, parity);
  else
    launch_cg_update(c, prec, parity);
  launch_precond_apply(c, prec, pc);
}

ms_status time_cg_spmv(ms_ctx* c, int prec, int reps, double* avg_us, double* bytes) {
  const int64_t ns = c->pat.nslices;
  const unsigned nbs = unsigned((ns + 3) / 4);
  MS_HIP(hipMemsetAsync(c->d_scal + S_DONE, 0, sizeof(double), c->stream));
  auto run = [&]() {
    with_slice(c->pat.S, [&](auto SS) {
      constexpr int S = decltype(SS)::value;
      if (prec == MS_PREC_FP64)
        k_cg_spmv<double, S><<<nbs, 256, 0, c->stream>>>(c->n, ns, c->pat.d_slice_base, c->pat.d_col, c->d_vals,
                                                         c->d_u, c->d_w, c->d_r, c->d_pinned, c->d_scal, c->d_part);
      else
        k_cg_spmv<float, S><<<nbs, 256, 0, c->stream>>>(c->n, ns, c->pat.d_slice_base, c->pat.d_col, c->d_vals32,
                                                        c->d_u, c->d_w, c->d_r, c->d_pinned, c->d_scal, c->d_part);
    });
  };
  for (int i = 0; i < 3; ++i) run();
  hipEvent_t e0, e1;
  MS_HIP(hipEventCreate(&e0));
  MS_HIP(hipEventCreate(&e1));
  MS_HIP(hipEventRecord(e0, c->stream));
  for (int i = 0; i < reps; ++i) run();
  MS_HIP(hipEventRecord(e1, c->stream));
  MS_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  MS_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_us = 1e3 * double(ms) / reps;
  *bytes = cg_spmv_bytes(c, prec);
  return MS_OK;
}

// Algorithmic bytes of one k_cg_spmv launch: 9 values + 1 column index per
// stored block, the slice offsets, u and r read and w written (FP64), the
// Dirichlet mask; padding lanes and the per-block partials are not counted.
double cg_spmv_bytes(const ms_ctx* c, int prec) {
  const double vb = prec == MS_PREC_FP64 ? 8.0 : 4.0;
  return double(c->pat.nnzb) * (9.0 * vb + 4.0) + 4.0 * double(c->pat.nslices + 1) +
         double(c->n) * (3.0 * 8.0 * 3.0 + 1.0);
}

// ---------------------------------------------------------------------------
// Standalone sliced-BSR3 matrix (SpMV measurements).
// ---------------------------------------------------------------------------
}  // namespace ms

namespace ms {
ms_status mat_build(ms_mat* A, int64_t n, const int32_t* row_ptr, const int32_t* col, const double* vals) {
  ms_ctx* c = &A->ctx;
  Pattern& P = c->pat;
  P.n = n;
  c->n = n;
  P.nnzb = row_ptr[n];
  for (int64_t b = 0; b < P.nnzb; ++b)
    if (col[b] < 0 || col[b] >= n) return fail(c, MS_E_ARG, "column index out of range");
  for (int64_t r = 0; r < n; ++r)
    if (row_ptr[r + 1] < row_ptr[r]) return fail(c, MS_E_ARG, "row_ptr not monotone");
  // slice height: MS_SLICE, else the fastest candidate on this pattern
  int S = 0;
  if (const char* e = std::getenv("MS_SLICE")) S = std::atoi(e);
  auto layout = [&](int cand, std::vector<int32_t>& sb, std::vector<int32_t>& sc, int& mw) {
    slice_layout(n, row_ptr, cand, sb, mw);
    sc.assign(sb.back(), -1);
    for (int64_t r = 0; r < n; ++r)
      for (int32_t k = 0; k < row_ptr[r + 1] - row_ptr[r]; ++k)
        sc[sb[r / cand] + int64_t(k) * cand + r % cand] = col[row_ptr[r] + k];
  };
  if (S != 16 && S != 32 && S != 64) {
    double best = 1e300;
    for (int cand : {16, 32, 64}) {
      std::vector<int32_t> sb, sc;
      int mw = 0;
      layout(cand, sb, sc, mw);
      int32_t *d_sb = nullptr, *d_sc = nullptr;
      ms_status st;
      if ((st = upload(c, &d_sb, sb.data(), sb.size())) || (st = upload(c, &d_sc, sc.data(), sc.size()))) return st;
      const double t = time_spmv_layout(c, cand, d_sb, d_sc, int64_t(sb.size()) - 1, sb.back(), 10);
      dfree(c, d_sb);
      dfree(c, d_sc);
      if (t < 0) return fail(c, MS_E_DEVICE, "SpMV layout timing failed");
      if (t < best) best = t, S = cand;
    }
  }
  P.S = S;
  std::vector<int32_t> scol;
  layout(S, P.h_slice_base, scol, P.maxw);
  P.nslices = int64_t(P.h_slice_base.size()) - 1;
  P.nslots = P.h_slice_base[P.nslices];
  const bool f32 = A->dtype == 1;
  std::vector<double> v64;
  std::vector<float> v32;
  if (f32)
    v32.assign(9 * P.nslots, 0.0f);
  else
    v64.assign(9 * P.nslots, 0.0);
  for (int64_t r = 0; r < n; ++r) {
    const int64_t s = r / S, lane = r % S;
    for (int32_t k = 0; k < row_ptr[r + 1] - row_ptr[r]; ++k) {
      const int64_t b = row_ptr[r] + k;
      const int64_t slot = P.h_slice_base[s] + int64_t(k) * S + lane;
      for (int cc = 0; cc < 9; ++cc) {
        const int64_t vi = vbase(slot, S) + int64_t(S) * cc;
        if (f32)
          v32[vi] = float(vals[9 * b + cc]);
        else
          v64[vi] = vals[9 * b + cc];
      }
    }
  }
  ms_status st;
  if ((st = upload(c, &P.d_slice_base, P.h_slice_base.data(), P.nslices + 1))) return st;
  if ((st = upload(c, &P.d_col, scol.data(), P.nslots))) return st;
  if (f32) {
    if ((st = upload(c, &c->d_vals32, v32.data(), v32.size()))) return st;
  } else {
    if ((st = upload(c, &c->d_vals, v64.data(), v64.size()))) return st;
  }
  const double vb = f32 ? 4.0 : 8.0;
  A->bytes = double(P.nnzb) * (9 * vb + 4) + 4.0 * double(P.nslices + 1) + 2.0 * 3 * n * vb;
  return MS_OK;
}

void mat_spmv(ms_mat* A, const void* x, void* y) {
  ms_ctx* c = &A->ctx;
  const int64_t ns = c->pat.nslices;
  with_slice(c->pat.S, [&](auto SS) {
    constexpr int S = decltype(SS)::value;
    if (A->dtype == 1)
      k_spmv<float, float, S><<<unsigned((ns + 3) / 4), 256, 0, c->stream>>>(
          c->n, ns, c->pat.d_slice_base, c->pat.d_col, c->d_vals32, static_cast<const float*>(x),
          static_cast<float*>(y), nullptr);
    else
      k_spmv<double, double, S><<<unsigned((ns + 3) / 4), 256, 0, c->stream>>>(
          c->n, ns, c->pat.d_slice_base, c->pat.d_col, c->d_vals, static_cast<const double*>(x),
          static_cast<double*>(y), nullptr);
  });
}
}  // namespace ms
