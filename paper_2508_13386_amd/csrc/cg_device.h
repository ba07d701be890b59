// Device pieces shared by the single-scene and the batched PCG kernels:
// sliced-BSR3 row products, the Chronopoulos-Gear scalar recurrence and the
// 3x3 block-Jacobi application.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ms_internal.h"

namespace ms {

// Row sums of y = A x for the rows of one slice (slots base .. base + width S)
// handled by this wave; lane = kq * S + r serves row r of the slice and
// block columns k = kq, kq + R, ... (R = 64 / S).  Columns are taken four at
// a time with every load of a batch issued before any is used (column
// index, nine values, three x entries), so the index -> x dependence costs
// one memory latency per batch instead of one per block.  Padding slots
// (column -1, zero values) and batch positions past the row end read x at
// column 0 and are weighted by zero.  Every lane of a row returns the full
// sum.
template <typename VT, typename XT, int S>
__device__ __forceinline__ void row_product_range(int base, int width, int lane, const int32_t* __restrict__ scol,
                                                  const VT* __restrict__ vals, const XT* __restrict__ x,
                                                  double y[3]) {
  constexpr int R = 64 / S;
  constexpr int NB = 4;
  const int r = lane % S, kq = lane / S;
  y[0] = y[1] = y[2] = 0.0;
  for (int k0 = kq; k0 < width; k0 += NB * R) {
    int64_t slot[NB];
    int col[NB];
    double f[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int k = k0 + u * R;
      slot[u] = int64_t(base) + int64_t(k < width ? k : k0) * S + r;
      col[u] = scol[slot[u]];
    }
    double a[NB][9], xv[NB][3];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int k = k0 + u * R;
      f[u] = (k < width && col[u] >= 0) ? 1.0 : 0.0;
      const int64_t cc = col[u] >= 0 ? col[u] : 0;
      const VT* ap = vals + vbase(slot[u], S);
#pragma unroll
      for (int q = 0; q < 9; ++q) a[u][q] = double(ap[q * S]);
#pragma unroll
      for (int q = 0; q < 3; ++q) xv[u][q] = double(x[3 * cc + q]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        y[i] += f[u] * (a[u][3 * i] * xv[u][0] + a[u][3 * i + 1] * xv[u][1] + a[u][3 * i + 2] * xv[u][2]);
  }
#pragma unroll
  for (int o = S; o < 64; o <<= 1)
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] += __shfl_xor(y[i], o, 64);
}

template <typename VT, typename XT, int S>
__device__ __forceinline__ void row_product(int64_t s, int lane, const int32_t* __restrict__ slice_base,
                                            const int32_t* __restrict__ scol, const VT* __restrict__ vals,
                                            const XT* __restrict__ x, double y[3]) {
  const int base = slice_base[s];
  row_product_range<VT, XT, S>(base, (slice_base[s + 1] - base) / S, lane, scol, vals, x, y);
}

enum { ST_GAMMA = 0, ST_ALPHA = 1, ST_ITER = 2, ST_N = 4 };

// Chronopoulos-Gear scalars from the dots (gamma = r.u, delta = w.u, rho =
// r.r).  Returns the done code (0 running, 1 converged, 2 iteration cap,
// 3 loss of positive definiteness).
__device__ __forceinline__ int cg_scalars(const double* st, const double* scal, double gamma, double delta,
                                          double rho, double& alpha, double& beta) {
  const double it = st[ST_ITER];
  alpha = beta = 0.0;
  if (rho <= scal[S_TOL2]) return 1;
  if (it >= scal[S_MAXIT]) return 2;
  if (it == 0.0 || st[ST_GAMMA] == 0.0) {
    beta = 0.0;
    alpha = gamma / delta;
  } else {
    beta = gamma / st[ST_GAMMA];
    alpha = gamma / (delta - beta * gamma / st[ST_ALPHA]);
  }
  if (!(alpha > 0.0) || !isfinite(alpha) || !isfinite(beta)) return 3;
  return 0;
}

// Block-Jacobi application u = Dinv r for one vertex.
template <typename VT>
__device__ __forceinline__ void bj_apply(const VT* __restrict__ Dinv, int64_t v, const double r[3], double u[3]) {
  const VT* D = Dinv + 9 * v;
  u[0] = double(D[0]) * r[0] + double(D[1]) * r[1] + double(D[2]) * r[2];
  u[1] = double(D[3]) * r[0] + double(D[4]) * r[1] + double(D[5]) * r[2];
  u[2] = double(D[6]) * r[0] + double(D[7]) * r[1] + double(D[8]) * r[2];
}

// Calls f(std::integral_constant<int, S>) for the runtime slice height.
template <typename F>
inline void with_slice(int S, F&& f) {
  if (S == 16)
    f(std::integral_constant<int, 16>());
  else if (S == 32)
    f(std::integral_constant<int, 32>());
  else
    f(std::integral_constant<int, 64>());
}

}  // namespace ms
