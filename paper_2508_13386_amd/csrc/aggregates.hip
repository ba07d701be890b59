// Aggregate block-Jacobi smoother for the Newton PCG (an option beside the
// 3x3 vertex blocks of the full-space block-Jacobi preconditioner; the
// paper's subspace solves use block-Jacobi per handle, Sec. 3.7.1).
//
// The stiff-contrast, nearly incompressible blocks this solver targets keep
// strong couplings between neighbouring vertices that 3x3 vertex blocks
// ignore.  Here vertices are grouped into compact aggregates of at most
// kAggV = 8 (2 x 2 x 2 on a regular grid) and the smoother applies the exact
// inverse of each aggregate's 24 x 24 diagonal block of H:
//   z = B^-1 r,  B = blockdiag_a(H_aa),
// in place of z = D^-1 r (D the 3x3 block diagonal).  B^-1 is symmetric
// positive definite whenever H is, so the additive two-level preconditioner
// z = B^-1 r + U (U^T H U)^-1 U^T r stays SPD.
//
//   aggregation   host, once per mesh pattern: rest positions binned into
//                 cubes of twice the shortest edge (offset by half an edge,
//                 so a regular grid falls into 2 x 2 x 2 blocks), each bin
//                 split in vertex order into groups of at most kAggV
//   k_agg_invert  per Newton iteration: one wave per aggregate gathers
//                 H_aa from the sliced BSR3 values, inverts it in FP64
//                 (Gauss-Jordan in LDS; SPD, no pivoting; pinned and padding
//                 DOFs as identity rows, zeroed afterwards), symmetrises,
//                 stores FP64 or FP32
//   k_cg_update_agg  the PCG update (k_cg_update's arithmetic) organised by
//                 aggregates, 32 lanes per aggregate (24 active), followed by
//                 u = B^-1 r_new from the aggregate's new residual in LDS
//   k_agg_apply   u = B^-1 r (start of each PCG solve)
#include <algorithm>
#include <array>
#include <cmath>
#include <type_traits>
#include <vector>

#include "cg_device.h"
#include "ms_internal.h"
#include "reduce.h"

namespace ms {

namespace {

constexpr int kAggLanes = 32;                     // lanes per aggregate in the update and apply kernels
constexpr int kAggPerBlock = kUpdBlock / kAggLanes;  // aggregates per 256-thread block
static_assert(kAggN <= kAggLanes, "one lane per aggregate DOF");

// One row of an aggregate inverse (kAggN entries, 16-byte aligned: rows start
// at multiples of kAggN entries) in 16-byte loads.
template <typename VT>
__device__ __forceinline__ void load_row(const VT* __restrict__ row, VT (&b)[kAggN]) {
  using V = typename std::conditional<sizeof(VT) == 4, float4, double2>::type;
  constexpr int W = 16 / sizeof(VT);
  static_assert(kAggN % W == 0, "whole 16-byte pieces");
#pragma unroll
  for (int q = 0; q < kAggN / W; ++q) {
    const V x = reinterpret_cast<const V*>(row)[q];
    const VT* px = reinterpret_cast<const VT*>(&x);
#pragma unroll
    for (int l = 0; l < W; ++l) b[W * q + l] = px[l];
  }
}

// Inverse of the aggregate blocks.  One 64-lane wave per aggregate.
template <typename VT>
__global__ void __launch_bounds__(64) k_agg_invert(int nagg, int S, const int32_t* __restrict__ vert,
                                                   const int32_t* __restrict__ slot, const VT* __restrict__ vals,
                                                   const uint8_t* __restrict__ pinned, double* __restrict__ inv64,
                                                   float* __restrict__ inv32) {
  __shared__ double A[kAggN][kAggN + 1];
  __shared__ double fcol[kAggN];
  __shared__ int act[kAggN];
  const int a = blockIdx.x, t = threadIdx.x;
  if (a >= nagg) return;
  if (t < kAggN) {
    const int v = vert[kAggV * a + t / 3];
    act[t] = (v >= 0 && !pinned[v]) ? 1 : 0;
  }
  __syncthreads();
  for (int e = t; e < kAggN * kAggN; e += 64) {
    const int i = e / kAggN, j = e % kAggN;
    double val;
    if (act[i] && act[j]) {
      const int s = slot[(kAggV * a + i / 3) * kAggV + j / 3];
      val = s >= 0 ? double(vals[vbase(s, S) + (3 * (i % 3) + j % 3) * S]) : 0.0;
    } else {
      val = i == j ? 1.0 : 0.0;
    }
    A[i][j] = val;
  }
  __syncthreads();
  // in-place Gauss-Jordan: after step k, column k holds the inverse's column
  for (int k = 0; k < kAggN; ++k) {
    const double pinv = 1.0 / A[k][k];
    if (t < kAggN) fcol[t] = A[t][k];
    __syncthreads();
    if (t < kAggN) A[k][t] = (t == k ? 1.0 : A[k][t]) * pinv;
    __syncthreads();
    for (int e = t; e < kAggN * kAggN; e += 64) {
      const int i = e / kAggN, j = e % kAggN;
      if (i == k) continue;
      A[i][j] = (j == k ? 0.0 : A[i][j]) - fcol[i] * A[k][j];
    }
    __syncthreads();
  }
  for (int e = t; e < kAggN * kAggN; e += 64) {
    const int i = e / kAggN, j = e % kAggN;
    const double z = (act[i] && act[j]) ? 0.5 * (A[i][j] + A[j][i]) : 0.0;
    const int64_t o = int64_t(a) * kAggN * kAggN + e;
    if (inv64) inv64[o] = z;
    if (inv32) inv32[o] = float(z);
  }
}

// u = B^-1 r.  32 lanes per aggregate, lane i < kAggN serves DOF i.
template <typename VT>
__global__ void __launch_bounds__(kUpdBlock) k_agg_apply(int nagg, const int32_t* __restrict__ vert,
                                                         const VT* __restrict__ inv, const double* __restrict__ r,
                                                         double* __restrict__ u) {
  __shared__ double rs[kAggPerBlock][kAggN];
  const int la = threadIdx.x / kAggLanes, i = threadIdx.x % kAggLanes;
  const int a = blockIdx.x * kAggPerBlock + la;
  const bool lane = i < kAggN && a < nagg;
  const int v = lane ? vert[kAggV * a + i / 3] : -1;
  const int64_t k = v >= 0 ? 3 * int64_t(v) + i % 3 : 0;
  if (lane) rs[la][i] = v >= 0 ? r[k] : 0.0;
  __syncthreads();
  if (v < 0) return;
  VT b[kAggN];
  load_row<VT>(inv + (int64_t(a) * kAggN + i) * kAggN, b);
  double z = 0.0;
#pragma unroll
  for (int j = 0; j < kAggN; ++j) z += double(b[j]) * rs[la][j];
  u[k] = z;
}

// The PCG update of k_cg_update (same partial reduction, scalars and
// expressions), by aggregates, then u = B^-1 r_new.  Every vertex belongs to
// exactly one aggregate, so every DOF is updated once.
template <typename VT>
__global__ void __launch_bounds__(kUpdBlock) k_cg_update_agg(int nagg, int nparts, const double* __restrict__ part,
                                                             const double* __restrict__ st_in,
                                                             double* __restrict__ st_out, double* __restrict__ p,
                                                             double* __restrict__ s, double* __restrict__ d,
                                                             double* __restrict__ r, double* __restrict__ u,
                                                             const double* __restrict__ w,
                                                             const int32_t* __restrict__ vert,
                                                             const VT* __restrict__ inv, double* __restrict__ scal) {
  __shared__ double rs[kAggPerBlock][kAggN];
  const double done = scal[S_DONE];
  const int la = threadIdx.x / kAggLanes, i = threadIdx.x % kAggLanes;
  const int a = blockIdx.x * kAggPerBlock + la;
  const bool lane = i < kAggN && a < nagg;
  const int v = lane ? vert[kAggV * a + i / 3] : -1;
  const bool own = v >= 0;
  const int64_t k = own ? 3 * int64_t(v) + i % 3 : 0;
  const double uo = u[k], po = p[k], wo = w[k], so = s[k], ro = r[k];
  VT b[kAggN];
  load_row<VT>(inv + (int64_t(lane ? a : 0) * kAggN + (lane ? i : 0)) * kAggN, b);
  if (done != 0.0) return;  // the flag is the same for the whole grid
  double dots[3] = {0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < nparts; q += blockDim.x)
#pragma unroll
    for (int c = 0; c < 3; ++c) dots[c] += part[3 * q + c];
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
  if (code != 0) return;
  double rr = 0.0;
  if (own) {
    const double pi = uo + beta * po;
    const double si = wo + beta * so;
    p[k] = pi;
    s[k] = si;
    d[k] += alpha * pi;
    rr = ro - alpha * si;
    r[k] = rr;
  }
  if (lane) rs[la][i] = rr;
  __syncthreads();
  if (!own) return;
  double z = 0.0;
#pragma unroll
  for (int j = 0; j < kAggN; ++j) z += double(b[j]) * rs[la][j];
  u[k] = z;
}

}  // namespace

// Vertex aggregates of a mesh: rest positions X [n][3] binned into cubes of
// twice the shortest edge of the vertex graph (CSR row_ptr / col, self
// entries allowed), the bins offset by half an edge so that a regular grid
// falls into 2 x 2 x 2 vertices; bins in (z, y, x) order, each split in
// vertex order into groups of at most kAggV.  vert receives kAggV entries
// per aggregate (vertex ids, -1 padding).
void aggregate_vertices(int64_t n, const double* X, const int32_t* row_ptr, const int32_t* col,
                        std::vector<int32_t>& vert) {
  double hmin = INFINITY, lo[3] = {INFINITY, INFINITY, INFINITY};
  for (int64_t v = 0; v < n; ++v) {
    for (int q = 0; q < 3; ++q) lo[q] = std::min(lo[q], X[3 * v + q]);
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      const int64_t j = col[e];
      if (j == v) continue;
      const double dx = X[3 * j] - X[3 * v], dy = X[3 * j + 1] - X[3 * v + 1], dz = X[3 * j + 2] - X[3 * v + 2];
      const double l = std::sqrt(dx * dx + dy * dy + dz * dz);
      if (l > 0.0) hmin = std::min(hmin, l);
    }
  }
  if (!std::isfinite(hmin)) hmin = 1.0;  // no edge of positive length
  std::vector<std::array<int64_t, 3>> key(n);
  for (int64_t v = 0; v < n; ++v)
    for (int q = 0; q < 3; ++q) key[v][q] = int64_t(std::floor((X[3 * v + q] - lo[q]) / (2.0 * hmin) + 0.25));
  std::vector<int64_t> order(n);
  for (int64_t v = 0; v < n; ++v) order[v] = v;
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    if (key[x][2] != key[y][2]) return key[x][2] < key[y][2];
    if (key[x][1] != key[y][1]) return key[x][1] < key[y][1];
    if (key[x][0] != key[y][0]) return key[x][0] < key[y][0];
    return x < y;
  });
  vert.clear();
  for (int64_t b = 0; b < n;) {
    int64_t e = b;
    while (e < n && key[order[e]] == key[order[b]]) ++e;
    for (int64_t g = b; g < e; g += kAggV)
      for (int q = 0; q < kAggV; ++q) vert.push_back(g + q < e ? int32_t(order[g + q]) : -1);
    b = e;
  }
}

// Aggregates of the context's mesh with the block slots of the current
// pattern, uploaded; inverse storage allocated.
ms_status build_aggregates(ms_ctx* c) {
  auto& G = c->agg;
  if (G.built) return MS_OK;
  const int64_t n = c->n;
  const Pattern& P = c->pat;
  if (n <= 0 || int64_t(P.h_row_ptr.size()) != n + 1) return fail(c, MS_E_ORDER, "upload a mesh first");
  if (P.nslots >= int64_t(1) << 31) return fail(c, MS_E_ARG, "too many block slots for the aggregate smoother");
  std::vector<int32_t> vert;
  aggregate_vertices(n, c->h_rest.data(), P.h_row_ptr.data(), P.h_col.data(), vert);
  const int nagg = int(vert.size() / kAggV);
  std::vector<int32_t> slot(size_t(nagg) * kAggV * kAggV, -1);
  for (int a = 0; a < nagg; ++a)
    for (int i = 0; i < kAggV; ++i) {
      const int32_t vi = vert[size_t(a) * kAggV + i];
      if (vi < 0) continue;
      const auto b0 = P.h_col.begin() + P.h_row_ptr[vi], b1 = P.h_col.begin() + P.h_row_ptr[vi + 1];
      for (int j = 0; j < kAggV; ++j) {
        const int32_t vj = vert[size_t(a) * kAggV + j];
        if (vj < 0) continue;
        const auto it = std::lower_bound(b0, b1, vj);
        if (it != b1 && *it == vj) slot[(size_t(a) * kAggV + i) * kAggV + j] = int32_t(P.h_slot_of_bsr[it - P.h_col.begin()]);
      }
    }
  ms_status s;
  if ((s = upload(c, &G.d_vert, vert.data(), vert.size())) || (s = upload(c, &G.d_slot, slot.data(), slot.size())) ||
      (s = alloc_n(c, &G.d_inv64, size_t(nagg) * kAggN * kAggN)) ||
      (s = alloc_n(c, &G.d_inv32, size_t(nagg) * kAggN * kAggN)))
    return s;
  G.nagg = nagg;
  G.built = true;
  return MS_OK;
}

void launch_agg_invert(ms_ctx* c, int prec) {
  auto& G = c->agg;
  if (prec == MS_PREC_FP64)
    k_agg_invert<double><<<unsigned(G.nagg), 64, 0, c->stream>>>(G.nagg, c->pat.S, G.d_vert, G.d_slot, c->d_vals,
                                                                 c->d_pinned, G.d_inv64, nullptr);
  else
    k_agg_invert<float><<<unsigned(G.nagg), 64, 0, c->stream>>>(G.nagg, c->pat.S, G.d_vert, G.d_slot, c->d_vals32,
                                                                c->d_pinned, nullptr, G.d_inv32);
}

void launch_agg_apply(ms_ctx* c, int prec) {
  auto& G = c->agg;
  const unsigned nb = unsigned((G.nagg + kAggPerBlock - 1) / kAggPerBlock);
  if (prec == MS_PREC_FP64)
    k_agg_apply<double><<<nb, kUpdBlock, 0, c->stream>>>(G.nagg, G.d_vert, G.d_inv64, c->d_r, c->d_u);
  else
    k_agg_apply<float><<<nb, kUpdBlock, 0, c->stream>>>(G.nagg, G.d_vert, G.d_inv32, c->d_r, c->d_u);
}

// `parity` as in launch_cg_update.
void launch_cg_update_agg(ms_ctx* c, int prec, int parity) {
  auto& G = c->agg;
  const unsigned nbs = unsigned((c->pat.nslices + 3) / 4);
  const unsigned nb = unsigned((G.nagg + kAggPerBlock - 1) / kAggPerBlock);
  const double* st_in = c->d_cgst + ST_N * parity;
  double* st_out = c->d_cgst + ST_N * (1 - parity);
  if (prec == MS_PREC_FP64)
    k_cg_update_agg<double><<<nb, kUpdBlock, 0, c->stream>>>(G.nagg, int(nbs), c->d_part, st_in, st_out, c->d_p,
                                                             c->d_s, c->d_d, c->d_r, c->d_u, c->d_w, G.d_vert,
                                                             G.d_inv64, c->d_scal);
  else
    k_cg_update_agg<float><<<nb, kUpdBlock, 0, c->stream>>>(G.nagg, int(nbs), c->d_part, st_in, st_out, c->d_p,
                                                            c->d_s, c->d_d, c->d_r, c->d_u, c->d_w, G.d_vert,
                                                            G.d_inv32, c->d_scal);
}

}  // namespace ms

extern "C" ms_status ms_aggregates_compute(int64_t n, const double* rest_xyz, const int32_t* row_ptr,
                                           const int32_t* col, int64_t cap, int32_t* vert, int64_t* n_agg) {
  if (n < 1 || !rest_xyz || !row_ptr || !col || !n_agg || cap < 0 || (cap > 0 && !vert)) return MS_E_ARG;
  if (row_ptr[0] != 0) return MS_E_MESH;
  for (int64_t v = 0; v < n; ++v) {
    if (row_ptr[v + 1] < row_ptr[v]) return MS_E_MESH;
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(rest_xyz[3 * v + q])) return MS_E_NONFINITE;
  }
  for (int64_t e = 0; e < row_ptr[n]; ++e)
    if (col[e] < 0 || col[e] >= n) return MS_E_MESH;
  std::vector<int32_t> out;
  ms::aggregate_vertices(n, rest_xyz, row_ptr, col, out);
  *n_agg = int64_t(out.size()) / ms::kAggV;
  if (cap > 0) std::copy(out.begin(), out.begin() + std::min<int64_t>(cap, int64_t(out.size())), vert);
  return MS_OK;
}
