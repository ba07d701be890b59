// Sparse products and preconditioned conjugate gradient for H d = -g
// (the Newton system of Sec. 3.1), on the sliced BSR3 layout.
//
// PCG uses the Chronopoulos-Gear recurrence, which needs one fused grid
// reduction per iteration: per iteration two kernels run,
//   k_cg_spmv    w = H u, the dots (r.u, w.u, r.r), and -- in the last block
//                to finish -- the scalar recurrences alpha, beta and the
//                convergence test, written to device memory;
//   k_cg_update  p = u + beta p, s = w + beta s, d += alpha p, r -= alpha s,
//                u = S r (3x3 block-Jacobi; the two-level preconditioner adds
//                its coarse correction in separate kernels).
// Every kernel returns at once when the device "done" flag is set, so fixed
// chunks of iterations can be captured in a HIP graph and replayed with one
// host synchronisation per chunk.
#include <algorithm>

#include "ms_internal.h"
#include "reduce.h"

namespace ms {

template <typename T>
struct Acc;
template <>
struct Acc<double> {
  using type = double;
};
template <>
struct Acc<float> {
  using type = float;
};

// y = A x, one wave per 64-row slice, one row per lane.
template <typename VT, typename XT>
__device__ __forceinline__ void row_product(int64_t s, int lane, const int32_t* __restrict__ slice_base,
                                            const int32_t* __restrict__ scol, const VT* __restrict__ vals,
                                            const XT* __restrict__ x, typename Acc<VT>::type y[3]) {
  using AT = typename Acc<VT>::type;
  const int base = slice_base[s];
  const int width = (slice_base[s + 1] - base) / kSlice;
  y[0] = y[1] = y[2] = AT(0);
  for (int k = 0; k < width; ++k) {
    const int64_t slot = int64_t(base) + int64_t(k) * kSlice + lane;
    const int col = scol[slot];
    if (col < 0) continue;
    const VT* a = vals + 9 * slot - 8 * lane;
    const AT x0 = AT(x[3 * int64_t(col)]), x1 = AT(x[3 * int64_t(col) + 1]), x2 = AT(x[3 * int64_t(col) + 2]);
    y[0] += AT(a[0]) * x0 + AT(a[64]) * x1 + AT(a[128]) * x2;
    y[1] += AT(a[192]) * x0 + AT(a[256]) * x1 + AT(a[320]) * x2;
    y[2] += AT(a[384]) * x0 + AT(a[448]) * x1 + AT(a[512]) * x2;
  }
}

template <typename VT, typename XT>
__global__ void __launch_bounds__(64) k_spmv(int64_t n, const int32_t* __restrict__ slice_base,
                                             const int32_t* __restrict__ scol, const VT* __restrict__ vals,
                                             const XT* __restrict__ x, XT* __restrict__ y,
                                             const uint8_t* __restrict__ pinned) {
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t row = s * kSlice + lane;
  typename Acc<VT>::type acc[3];
  row_product<VT, XT>(s, lane, slice_base, scol, vals, x, acc);
  if (row < n) {
    const bool pin = pinned && pinned[row];
    y[3 * row] = pin ? XT(0) : XT(acc[0]);
    y[3 * row + 1] = pin ? XT(0) : XT(acc[1]);
    y[3 * row + 2] = pin ? XT(0) : XT(acc[2]);
  }
}

// ---------------------------------------------------------------------------
// PCG kernels.  VT: matrix / iteration vector type (double or float); the
// solution d and all dot products are accumulated in double.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void finalize_cg(double* scal, double gamma, double delta, double rho) {
  const double it = scal[S_ITER];
  if (rho <= scal[S_TOL2]) {
    scal[S_DONE] = 1.0;
    scal[S_RHO] = rho;
    return;
  }
  if (it >= scal[S_MAXIT]) {
    scal[S_DONE] = 2.0;
    scal[S_RHO] = rho;
    return;
  }
  double alpha, beta;
  if (it == 0.0 || scal[S_GAMMA_OLD] == 0.0) {
    beta = 0.0;
    alpha = gamma / delta;
  } else {
    beta = gamma / scal[S_GAMMA_OLD];
    alpha = gamma / (delta - beta * gamma / scal[S_ALPHA_OLD]);
  }
  if (!(alpha > 0.0) || !isfinite(alpha) || !isfinite(beta)) {  // loss of positive definiteness
    scal[S_DONE] = 3.0;
    scal[S_RHO] = rho;
    return;
  }
  scal[S_ALPHA] = alpha;
  scal[S_BETA] = beta;
  scal[S_ALPHA_OLD] = alpha;
  scal[S_GAMMA_OLD] = gamma;
  scal[S_RHO] = rho;
  scal[S_ITER] = it + 1.0;
}

template <typename VT>
__global__ void __launch_bounds__(64) k_cg_spmv(int64_t n, const int32_t* __restrict__ slice_base,
                                                const int32_t* __restrict__ scol, const VT* __restrict__ vals,
                                                const VT* __restrict__ u, VT* __restrict__ w,
                                                const VT* __restrict__ r, const uint8_t* __restrict__ pinned,
                                                double* __restrict__ scal, double* __restrict__ part,
                                                unsigned* __restrict__ counter) {
  if (scal[S_DONE] != 0.0) return;
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t row = s * kSlice + lane;
  typename Acc<VT>::type acc[3];
  row_product<VT, VT>(s, lane, slice_base, scol, vals, u, acc);
  double dots[3] = {0.0, 0.0, 0.0};
  if (row < n) {
    const bool pin = pinned[row];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const VT wi = pin ? VT(0) : VT(acc[i]);
      w[3 * row + i] = wi;
      const double ui = double(u[3 * row + i]), ri = double(r[3 * row + i]);
      dots[0] += ri * ui;
      dots[1] += double(wi) * ui;
      dots[2] += ri * ri;
    }
  }
  if (grid_sum<3>(dots, part, counter) && threadIdx.x == 0) finalize_cg(scal, dots[0], dots[1], dots[2]);
}

// Block-Jacobi application u = Dinv r for one vertex.
template <typename VT>
__device__ __forceinline__ void bj_apply(const VT* __restrict__ Dinv, int64_t v, const VT r[3], VT u[3]) {
  const VT* D = Dinv + 9 * v;
  u[0] = D[0] * r[0] + D[1] * r[1] + D[2] * r[2];
  u[1] = D[3] * r[0] + D[4] * r[1] + D[5] * r[2];
  u[2] = D[6] * r[0] + D[7] * r[1] + D[8] * r[2];
}

template <typename VT>
__global__ void __launch_bounds__(256) k_cg_update(int64_t n, VT* __restrict__ p, VT* __restrict__ s,
                                                   double* __restrict__ d, VT* __restrict__ r,
                                                   VT* __restrict__ u, const VT* __restrict__ w,
                                                   const VT* __restrict__ Dinv, const double* __restrict__ scal) {
  if (scal[S_DONE] != 0.0) return;
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double alpha = scal[S_ALPHA], beta = scal[S_BETA];
  VT rr[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int64_t k = 3 * v + i;
    const VT pi = VT(double(u[k]) + beta * double(p[k]));
    const VT si = VT(double(w[k]) + beta * double(s[k]));
    p[k] = pi;
    s[k] = si;
    d[k] += alpha * double(pi);
    rr[i] = VT(double(r[k]) - alpha * double(si));
    r[k] = rr[i];
  }
  VT uu[3];
  bj_apply<VT>(Dinv, v, rr, uu);
#pragma unroll
  for (int i = 0; i < 3; ++i) u[3 * v + i] = uu[i];
}

// d = 0, r = -g (zero on pinned DOFs), u = S r, p = s = 0; rho0 = r.r and the
// PCG scalars are initialised in the last block, with the forcing term
// eta = clamp(sqrt(||g|| / ||g_first||), eta_min, eta_max) of this Newton
// iteration.
template <typename VT>
__global__ void __launch_bounds__(256) k_cg_init(int64_t n, const double* __restrict__ g,
                                                 const uint8_t* __restrict__ pinned, VT* __restrict__ p,
                                                 VT* __restrict__ s, double* __restrict__ d, VT* __restrict__ r,
                                                 VT* __restrict__ u, const VT* __restrict__ Dinv, double eta_max,
                                                 double eta_min, int first, double maxit, double* __restrict__ scal,
                                                 double* __restrict__ part,
                                                 unsigned* __restrict__ counter) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double rho[1] = {0.0};
  if (v < n) {
    const bool pin = pinned[v];
    VT rr[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int64_t k = 3 * v + i;
      const double gi = pin ? 0.0 : -g[k];
      rr[i] = VT(gi);
      r[k] = rr[i];
      p[k] = VT(0);
      s[k] = VT(0);
      d[k] = 0.0;
      rho[0] += gi * gi;
    }
    VT uu[3];
    bj_apply<VT>(Dinv, v, rr, uu);
#pragma unroll
    for (int i = 0; i < 3; ++i) u[3 * v + i] = uu[i];
  }
  if (grid_sum<1>(rho, part, counter) && threadIdx.x == 0) {
    scal[S_RHO0] = rho[0];
    scal[S_RHO] = rho[0];
    if (first) scal[S_G0SQ] = rho[0];
    double eta = scal[S_G0SQ] > 0.0 ? sqrt(sqrt(rho[0] / scal[S_G0SQ])) : 1.0;
    eta = fmin(eta_max, fmax(eta_min, eta));
    scal[S_TOL2] = eta * eta * rho[0];
    scal[S_ITER] = 0.0;
    scal[S_MAXIT] = maxit;
    scal[S_GAMMA_OLD] = 0.0;
    scal[S_ALPHA_OLD] = 1.0;
    scal[S_DONE] = rho[0] > 0.0 ? 0.0 : 1.0;
  }
}

// Inverse of each diagonal 3x3 block (cofactor formula in double); pinned
// vertices get a zero block so that the preconditioned vectors vanish there.
template <typename VT>
__global__ void k_block_jacobi(int64_t n, const int32_t* __restrict__ diag_slot, const VT* __restrict__ vals,
                               const uint8_t* __restrict__ pinned, VT* __restrict__ Dinv) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t slot = diag_slot[v];
  const VT* a = vals + 9 * slot - 8 * (slot & 63);
  double m[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) m[c] = double(a[64 * c]);
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
__global__ void k_extract(int64_t nnzb, const int64_t* __restrict__ slot_of, const VT* __restrict__ vals,
                          double* __restrict__ out) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= nnzb) return;
  const int64_t slot = slot_of[b];
  const VT* a = vals + 9 * slot - 8 * (slot & 63);
#pragma unroll
  for (int c = 0; c < 9; ++c) out[9 * b + c] = double(a[64 * c]);
}

static inline unsigned nblocks(int64_t n, int b) { return unsigned((n + b - 1) / b); }

void launch_spmv(ms_ctx* c, int prec, const double* x, double* y) {
  // FP64 vectors; the FP32 matrix variant converts on load
  if (prec == MS_PREC_FP64)
    k_spmv<double, double><<<unsigned(c->pat.nslices), 64, 0, c->stream>>>(c->n, c->pat.d_slice_base, c->pat.d_col,
                                                                          c->d_vals, x, y, nullptr);
  else
    k_spmv<float, double><<<unsigned(c->pat.nslices), 64, 0, c->stream>>>(c->n, c->pat.d_slice_base, c->pat.d_col,
                                                                         c->d_vals32, x, y, nullptr);
}

void launch_block_jacobi(ms_ctx* c, int prec) {
  if (prec == MS_PREC_FP64)
    k_block_jacobi<double><<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, c->pat.d_diag_slot, c->d_vals,
                                                                     c->d_pinned, c->d_Dinv);
  else
    k_block_jacobi<float><<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, c->pat.d_diag_slot, c->d_vals32,
                                                                    c->d_pinned, c->d_Dinv32);
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
    k_extract<double><<<nblocks(nnzb, 256), 256, 0, c->stream>>>(nnzb, slot_of, c->d_vals, out);
  else
    k_extract<float><<<nblocks(nnzb, 256), 256, 0, c->stream>>>(nnzb, slot_of, c->d_vals32, out);
}

void launch_cg_init(ms_ctx* c, int prec, double eta_max, double eta_min, bool first, int max_it) {
  const unsigned nb = nblocks(c->n, 256);
  if (prec == MS_PREC_FP64)
    k_cg_init<double><<<nb, 256, 0, c->stream>>>(c->n, c->d_g, c->d_pinned, c->d_p, c->d_s, c->d_d, c->d_r, c->d_u,
                                                 c->d_Dinv, eta_max, eta_min, first ? 1 : 0, double(max_it), c->d_scal, c->d_part,
                                                 c->d_counter);
  else
    k_cg_init<float><<<nb, 256, 0, c->stream>>>(c->n, c->d_g, c->d_pinned, c->f_p, c->f_s, c->d_d, c->f_r, c->f_u,
                                                c->d_Dinv32, eta_max, eta_min, first ? 1 : 0, double(max_it), c->d_scal, c->d_part,
                                                c->d_counter);
}

void launch_cg_iteration(ms_ctx* c, int prec, int pc) {
  const unsigned ns = unsigned(c->pat.nslices), nb = nblocks(c->n, 256);
  if (prec == MS_PREC_FP64) {
    k_cg_spmv<double><<<ns, 64, 0, c->stream>>>(c->n, c->pat.d_slice_base, c->pat.d_col, c->d_vals, c->d_u, c->d_w,
                                                c->d_r, c->d_pinned, c->d_scal, c->d_part, c->d_counter);
    k_cg_update<double><<<nb, 256, 0, c->stream>>>(c->n, c->d_p, c->d_s, c->d_d, c->d_r, c->d_u, c->d_w, c->d_Dinv,
                                                   c->d_scal);
  } else {
    k_cg_spmv<float><<<ns, 64, 0, c->stream>>>(c->n, c->pat.d_slice_base, c->pat.d_col, c->d_vals32, c->f_u, c->f_w,
                                               c->f_r, c->d_pinned, c->d_scal, c->d_part, c->d_counter);
    k_cg_update<float><<<nb, 256, 0, c->stream>>>(c->n, c->f_p, c->f_s, c->d_d, c->f_r, c->f_u, c->f_w, c->d_Dinv32,
                                                  c->d_scal);
  }
  if (pc == MS_PC_TWO_LEVEL) launch_coarse_correction(c, prec);
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
  P.nnzb = row_ptr[n];
  P.nslices = (n + kSlice - 1) / kSlice;
  P.h_slice_base.assign(P.nslices + 1, 0);
  for (int64_t s = 0; s < P.nslices; ++s) {
    int32_t w = 0;
    for (int64_t r = s * kSlice; r < std::min<int64_t>(n, (s + 1) * kSlice); ++r)
      w = std::max(w, row_ptr[r + 1] - row_ptr[r]);
    P.h_slice_base[s + 1] = P.h_slice_base[s] + w * kSlice;
  }
  P.nslots = P.h_slice_base[P.nslices];
  std::vector<int32_t> scol(P.nslots, -1);
  const bool f32 = A->dtype == 1;
  std::vector<double> v64;
  std::vector<float> v32;
  if (f32)
    v32.assign(9 * P.nslots, 0.0f);
  else
    v64.assign(9 * P.nslots, 0.0);
  for (int64_t r = 0; r < n; ++r) {
    const int64_t s = r / kSlice, lane = r % kSlice;
    for (int32_t k = 0; k < row_ptr[r + 1] - row_ptr[r]; ++k) {
      const int64_t b = row_ptr[r] + k;
      if (col[b] < 0 || col[b] >= n) return fail(c, MS_E_ARG, "column index out of range");
      const int64_t slot = P.h_slice_base[s] + int64_t(k) * kSlice + lane;
      scol[slot] = col[b];
      for (int cc = 0; cc < 9; ++cc) {
        const int64_t vi = 9 * slot - 8 * lane + 64 * cc;
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
  c->n = n;
  return MS_OK;
}

void mat_spmv(ms_mat* A, const void* x, void* y) {
  ms_ctx* c = &A->ctx;
  if (A->dtype == 1)
    k_spmv<float, float><<<unsigned(c->pat.nslices), 64, 0, c->stream>>>(
        c->n, c->pat.d_slice_base, c->pat.d_col, c->d_vals32, static_cast<const float*>(x), static_cast<float*>(y),
        nullptr);
  else
    k_spmv<double, double><<<unsigned(c->pat.nslices), 64, 0, c->stream>>>(
        c->n, c->pat.d_slice_base, c->pat.d_col, c->d_vals, static_cast<const double*>(x),
        static_cast<double*>(y), nullptr);
}
}  // namespace ms
