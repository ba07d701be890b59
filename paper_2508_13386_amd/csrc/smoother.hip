// l1-scaled 3x3 block-Jacobi smoother of the symmetric two-level V(1,1)
// preconditioner (the full-space block-Jacobi level of the method, Sec. 5,
// used as pre- and post-smoother around the coarse correction on the sparse
// basis).  For vertex v the block D_vv + diag(l) is inverted, where l_i is
// the sum of |H_ij| over the row's off-diagonal blocks at free vertices; this
// bounds the spectrum of L H below 2 so that the V-cycle stays SPD for any
// SPD coarse matrix (also one that lags the Hessian).
#include "cg_device.h"
#include "ms_internal.h"

namespace ms {

template <typename VT, int S>
__global__ void __launch_bounds__(256) k_block_jacobi_l1(int64_t n, const int32_t* __restrict__ slice_base,
                                                         const int32_t* __restrict__ scol,
                                                         const int32_t* __restrict__ diag_slot,
                                                         const VT* __restrict__ vals,
                                                         const uint8_t* __restrict__ pinned, VT* __restrict__ Dinv) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t sl = v / S;
  const int lane = int(v % S);
  const int base = slice_base[sl], width = (slice_base[sl + 1] - base) / S;
  const int64_t dslot = diag_slot[v];
  double l1[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < width; ++k) {
    const int64_t slot = int64_t(base) + int64_t(k) * S + lane;
    const int col = scol[slot];
    if (col < 0 || slot == dslot || pinned[col]) continue;
    const VT* a = vals + vbase(slot, S);
#pragma unroll
    for (int i = 0; i < 3; ++i)
      l1[i] += fabs(double(a[S * (3 * i)])) + fabs(double(a[S * (3 * i + 1)])) + fabs(double(a[S * (3 * i + 2)]));
  }
  const VT* a = vals + vbase(dslot, S);
  double m[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) m[q] = double(a[S * q]);
  m[0] += l1[0];
  m[4] += l1[1];
  m[8] += l1[2];
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
  const double id = pinned[v] ? 0.0 : 1.0 / det;
#pragma unroll
  for (int q = 0; q < 9; ++q) Dinv[9 * v + q] = VT(inv[q] * id);
}

// u += L w (zero rows at pinned vertices come from their zero blocks).
template <typename VT>
__global__ void __launch_bounds__(256) k_bj_add(int64_t n, const double* __restrict__ w, double* __restrict__ u,
                                                const VT* __restrict__ Dinv, const double* __restrict__ scal) {
  if (scal && scal[S_DONE] != 0.0) return;
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double ww[3] = {w[3 * v], w[3 * v + 1], w[3 * v + 2]};
  double z[3];
  bj_apply<VT>(Dinv, v, ww, z);
#pragma unroll
  for (int i = 0; i < 3; ++i) u[3 * v + i] += z[i];
}

static inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

void launch_block_jacobi_l1(ms_ctx* c, int prec) {
  with_slice(c->pat.S, [&](auto SS) {
    constexpr int S = decltype(SS)::value;
    if (prec == MS_PREC_FP64)
      k_block_jacobi_l1<double, S><<<nblk(c->n, 256), 256, 0, c->stream>>>(
          c->n, c->pat.d_slice_base, c->pat.d_col, c->pat.d_diag_slot, c->d_vals, c->d_pinned, c->d_Dinv);
    else
      k_block_jacobi_l1<float, S><<<nblk(c->n, 256), 256, 0, c->stream>>>(
          c->n, c->pat.d_slice_base, c->pat.d_col, c->pat.d_diag_slot, c->d_vals32, c->d_pinned, c->d_Dinv32);
  });
}

void launch_bj_add(ms_ctx* c, int prec) {
  if (prec == MS_PREC_FP64)
    k_bj_add<double><<<nblk(c->n, 256), 256, 0, c->stream>>>(c->n, c->d_w, c->d_u, c->d_Dinv, c->d_scal);
  else
    k_bj_add<float><<<nblk(c->n, 256), 256, 0, c->stream>>>(c->n, c->d_w, c->d_u, c->d_Dinv32, c->d_scal);
}

}  // namespace ms
