// Two-level preconditioner built on the sparse material-aware basis U of
// Eq. (LBS): the columns of U at vertex v are phi_vi (I_3 (x) [1, x_v - o_i]).
//
//   restriction   c = U^T r          one block per handle, fixed-order sums
//   coarse solve  e = (U^T H U)^-1 c  explicit inverse of the Galerkin matrix
//                                     (FP64 Gauss-Jordan), applied as a GEMV
//                                     (FP32 copy in mixed precision)
//   prolongation  u += U e            8 lanes per vertex
// The PCG preconditioner is additive: z = D^-1 r + U (U^T H U)^-1 U^T r with
// D the 3x3 block diagonal of H (Sec. 3.7.1 uses the same triple product
// U^T H U matrix-free; here it is formed once per Newton iteration).
//
// Galerkin product in two atomic-free stages:
//   Z_vj[a][b][l] = sum_{w in N(v), j in h(w)} H_vw[a][b] W_wj[l]     (Z = H U)
//   A_(i,a,k),(j,b,l) = sum_{v: i in h(v)} W_vi[k] Z_vj[a][b][l]     (U^T Z)
// with W_vi = phi_vi [1, x_v - o_i]; both stages sum in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <chrono>
#include <map>
#include <type_traits>

#include "contact.h"
#include "ms_internal.h"
#include "reduce.h"

namespace ms {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_sub(int64_t len, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < len) out[i] = a[i] - b[i];
}

// Restriction partials of c = U^T (weight .* v).  One block of kRThreads
// threads per chunk of at most kRChunk entries of one handle's vertex list
// (entries in handle order: vertex hv[e] and weights hw[e] = W_vi, so the
// weight loads are contiguous); each thread takes kREnt entries with every
// load issued before any is used (clamped index, zero scale past the chunk
// end).
// The chunk's 12 sums are reduced in a fixed order and stored as a partial;
// the coarse GEMV adds a handle's partials in chunk order (no inter-block
// communication, hence no device-scope fences).
constexpr int kRChunk = 1024;
constexpr int kRThreads = 64;
constexpr int kREnt = kRChunk / kRThreads;
__global__ void __launch_bounds__(kRThreads) k_restrict(const int4* __restrict__ chunk_info, const int32_t* __restrict__ hv,
                                                  const double* __restrict__ hw, const double* __restrict__ v,
                                                  const double* __restrict__ weight, double* __restrict__ part,
                                                  const double* __restrict__ scal) {
  const int ch = blockIdx.x, t = threadIdx.x;
  const int4 info = chunk_info[ch];  // {handle, first entry, end entry, unused}
  const double done = scal ? scal[S_DONE] : 0.0;
  const int e0 = info.y, e1 = info.z;
  int vv[kREnt];
  double w[kREnt][4], sc[kREnt];
#pragma unroll
  for (int u = 0; u < kREnt; ++u) {
    const int e = e0 + t + kRThreads * u;
    const bool ok = e < e1;
    const int ec = ok ? e : 0;
    vv[u] = hv[ec];
    const double2 wa = *reinterpret_cast<const double2*>(hw + 4 * int64_t(ec));
    const double2 wb = *reinterpret_cast<const double2*>(hw + 4 * int64_t(ec) + 2);
    w[u][0] = wa.x;
    w[u][1] = wa.y;
    w[u][2] = wb.x;
    w[u][3] = wb.y;
    sc[u] = ok ? 1.0 : 0.0;
  }
  if (done != 0.0) return;  // the flag is the same for the whole grid
  double rv[kREnt][3];
#pragma unroll
  for (int u = 0; u < kREnt; ++u)
#pragma unroll
    for (int a = 0; a < 3; ++a) rv[u][a] = v[3 * int64_t(vv[u]) + a];
  if (weight)
#pragma unroll
    for (int u = 0; u < kREnt; ++u) sc[u] *= weight[vv[u]];
  double acc[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) acc[q] = 0.0;
#pragma unroll
  for (int u = 0; u < kREnt; ++u)
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const double wl = sc[u] * w[u][l];
      acc[l] += wl * rv[u][0];
      acc[4 + l] += wl * rv[u][1];
      acc[8 + l] += wl * rv[u][2];
    }
  block_sum<12>(acc);
  if (t < 12) {
    double out = 0.0;
#pragma unroll
    for (int q = 0; q < 12; ++q)
      if (t == q) out = acc[q];
    part[12 * int64_t(ch) + t] = out;
  }
}

// e = A c for a dense row-major r x r matrix A (FP64, or its FP32 copy in
// mixed precision; leading dimension ld a multiple of 4, rows readable up to
// ld) with c given by the restriction partials: every block first forms c in
// LDS (c_(12 i + q) = sum of handle i's partials q, in chunk order), then one
// wave per row, 16 rows per 1024-thread block.  The first kGemvPre 16-byte
// pieces of each lane's share of the row are loaded before the flag test
// and the formation of c, so their latency overlaps both.
constexpr int kGemvRows = 16;
static_assert(kGemvRows == kGemvRowsPerBlock, "the batched GEMV tables assume this row count");
constexpr int kGemvPre = 10;
// direct != 0: every handle's restriction is a single chunk and chunk i is
// handle i, so the partials are the coarse right-hand side itself; they are
// then loaded together with the matrix rows, before the flag test.
constexpr int kGemvPart = 3;  // direct loads per thread (r <= 3 * 64 * kGemvRows)
template <typename AT>
using V16T = typename std::conditional<sizeof(AT) == 4, float4, double2>::type;

// The first kGemvPre 16-byte pieces of this lane's share of row a.
template <typename AT>
__device__ __forceinline__ void gemv_preload(const AT* __restrict__ a, int ld, int lane, V16T<AT> (&pre)[kGemvPre]) {
  constexpr int VW = 16 / sizeof(AT);  // elements per 16-byte load
  constexpr int STRIDE = 64 * VW;
#pragma unroll
  for (int p = 0; p < kGemvPre; ++p) {
    const int j = VW * lane + STRIDE * p;
    pre[p] = j < ld ? *reinterpret_cast<const V16T<AT>*>(a + j) : V16T<AT>{};
  }
}

// sum_j a_j c_j over the r columns of one row, by one wave: the preloaded
// pieces first, then the rest of the lane's share, then a fixed-order wave
// reduction.
template <typename AT>
__device__ __forceinline__ double gemv_row(const AT* __restrict__ a, int r, int lane,
                                           const V16T<AT> (&pre)[kGemvPre], const double* sc) {
  constexpr int VW = 16 / sizeof(AT);
  constexpr int STRIDE = 64 * VW;
  double s = 0.0;
#pragma unroll
  for (int p = 0; p < kGemvPre; ++p) {
    const int j = VW * lane + STRIDE * p;
    const AT* pv = reinterpret_cast<const AT*>(&pre[p]);
#pragma unroll
    for (int q = 0; q < VW; ++q)
      if (j + q < r) s += double(pv[q]) * sc[j + q];
  }
  for (int j = VW * lane + STRIDE * kGemvPre; j < r; j += STRIDE) {
#pragma unroll
    for (int q = 0; q < VW; ++q)
      if (j + q < r) s += double(a[j + q]) * sc[j + q];
  }
  return wave_sum(s);
}

template <typename AT>
__global__ void __launch_bounds__(64 * kGemvRows) k_coarse_gemv(int r, int ld, const AT* __restrict__ A,
                                                      const int2* __restrict__ hinfo,
                                                      const double* __restrict__ part, double* __restrict__ e,
                                                      const double* __restrict__ scal, int direct) {
  extern __shared__ double sc[];
  const double done = scal ? scal[S_DONE] : 0.0;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int row = blockIdx.x * kGemvRows + wave;
  const AT* a = A + int64_t(row < r ? row : 0) * ld;
  double pc[kGemvPart];
  if (direct) {
#pragma unroll
    for (int u = 0; u < kGemvPart; ++u) {
      const int idx = t + u * int(blockDim.x);
      pc[u] = idx < r ? part[idx] : 0.0;
    }
  }
  V16T<AT> pre[kGemvPre];
  gemv_preload<AT>(a, ld, lane, pre);
  if (done != 0.0) return;  // the flag is the same for the whole grid
  if (direct) {
#pragma unroll
    for (int u = 0; u < kGemvPart; ++u) {
      const int idx = t + u * int(blockDim.x);
      if (idx < r) sc[idx] = pc[u];
    }
  } else {
    for (int idx = t; idx < r; idx += blockDim.x) {
      const int2 hi = hinfo[idx / 12];
      const int q = idx % 12;
      double s = 0.0;
      for (int k = 0; k < hi.y; ++k) s += part[12 * int64_t(hi.x + k) + q];
      sc[idx] = s;
    }
  }
  __syncthreads();
  if (row >= r) return;
  const double s = gemv_row<AT>(a, r, lane, pre, sc);
  if (lane == 0) e[row] = s;
}

// Block-diagonal e = A c over several scenes (the batched two-level
// preconditioner): block b serves kGemvRows rows of one scene, whose inverse
// (leading dimension ld, coarse size r) and handles (from union handle h0)
// its descriptor gives; c comes from the union's restriction partials.  The
// row arithmetic is k_coarse_gemv's, so every scene gets the values of its
// own unbatched preconditioner.
template <typename AT>
__global__ void __launch_bounds__(64 * kGemvRows) k_coarse_gemv_seg(const GemvSeg* __restrict__ seg,
                                                          const int2* __restrict__ hinfo,
                                                          const double* __restrict__ part, double* __restrict__ e,
                                                          const double* __restrict__ sscal, int sstride, int direct) {
  extern __shared__ double sc[];
  const GemvSeg g = seg[blockIdx.x];
  const double done = sscal ? sscal[int64_t(sstride) * g.scene + S_DONE] : 0.0;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int row = g.row0 + wave;
  const AT* A = static_cast<const AT*>(g.A);
  const AT* a = A + int64_t(row < g.r ? row : 0) * g.ld;
  V16T<AT> pre[kGemvPre];
  gemv_preload<AT>(a, g.ld, lane, pre);
  if (done != 0.0) return;  // the flag is the same for every block of the scene
  for (int idx = t; idx < g.r; idx += blockDim.x) {
    if (direct) {
      sc[idx] = part[12 * int64_t(g.h0) + idx];  // union chunk i is union handle i
    } else {
      const int2 hi = hinfo[g.h0 + idx / 12];
      const int q = idx % 12;
      double s = 0.0;
      for (int k = 0; k < hi.y; ++k) s += part[12 * int64_t(hi.x + k) + q];
      sc[idx] = s;
    }
  }
  __syncthreads();
  if (row >= g.r) return;
  const double s = gemv_row<AT>(a, g.r, lane, pre, sc);
  if (lane == 0) e[12 * int64_t(g.h0) + row] = s;
}

void launch_coarse_gemv_seg(ms_ctx* u, int prec, const GemvSeg* seg, int nblocks_seg, int rmax, const double* sscal,
                            int sstride) {
  Basis& D = u->basis;
  const int direct = D.nrchunks == D.m ? 1 : 0;
  const size_t lds = size_t(rmax) * sizeof(double);
  if (prec == MS_PREC_MIXED)
    k_coarse_gemv_seg<float><<<unsigned(nblocks_seg), 64 * kGemvRows, lds, u->stream>>>(seg, D.d_hinfo, D.d_rpart,
                                                                                       u->d_e, sscal, sstride, direct);
  else
    k_coarse_gemv_seg<double><<<unsigned(nblocks_seg), 64 * kGemvRows, lds, u->stream>>>(seg, D.d_hinfo, D.d_rpart,
                                                                                        u->d_e, sscal, sstride, direct);
}

// e = A c for a dense row-major r x r matrix (leading dimension ld), one
// wave per row.
__global__ void __launch_bounds__(256) k_gemv(int r, int ld, const double* __restrict__ A,
                                              const double* __restrict__ c, double* __restrict__ e,
                                              const double* __restrict__ scal) {
  if (scal && scal[S_DONE] != 0.0) return;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= r) return;
  double s = 0.0;
  const double* a = A + int64_t(row) * ld;
  for (int j = lane; j < r; j += 64) s += a[j] * c[j];
  s = wave_sum(s);
  if (lane == 0) e[row] = s;
}

// u_v += sum_i W_vi (x) e_i with 8 lanes per vertex (entry j of the vertex on
// lane j mod 8), reduced across the 8 lanes in a fixed order.
__global__ void __launch_bounds__(256) k_prolong8(int64_t n, const int32_t* __restrict__ vptr,
                                                  const int32_t* __restrict__ vh, const double* __restrict__ vw,
                                                  const double* __restrict__ e, const uint8_t* __restrict__ pinned,
                                                  double* __restrict__ u, const double* __restrict__ scal) {
  const double done = scal ? scal[S_DONE] : 0.0;
  const int64_t v = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 3;
  const int j = threadIdx.x & 7;
  const int64_t vc = v < n ? v : 0;
  const bool active = v < n && !(pinned && pinned[vc]);
  const int k0 = vptr[vc], k1 = vptr[vc + 1];
  const double uo = u[3 * vc + (j < 3 ? j : 0)];
  // first entry of this lane, loads issued unconditionally (clamped)
  const int kf = k0 + j;
  const int kc = kf < k1 ? kf : 0;
  const int hf = vh[kc];
  const double2 wa = *reinterpret_cast<const double2*>(vw + 4 * int64_t(kc));
  const double2 wb = *reinterpret_cast<const double2*>(vw + 4 * int64_t(kc) + 2);
  if (done != 0.0) return;  // the flag is the same for the whole grid
  double a[3] = {0.0, 0.0, 0.0};
  {
    const double fw = (active && kf < k1) ? 1.0 : 0.0;
    const double w[4] = {fw * wa.x, fw * wa.y, fw * wb.x, fw * wb.y};
    const double* q = e + 12 * int64_t(hf);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      a[0] += w[l] * q[l];
      a[1] += w[l] * q[4 + l];
      a[2] += w[l] * q[8 + l];
    }
  }
  if (active)
    for (int k = kf + 8; k < k1; k += 8) {  // vertices with more than 8 handles
      const double* wk = vw + 4 * int64_t(k);
      const double* q = e + 12 * int64_t(vh[k]);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        a[0] += wk[l] * q[l];
        a[1] += wk[l] * q[4 + l];
        a[2] += wk[l] * q[8 + l];
      }
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) a[i] += __shfl_xor(a[i], o, 64);
  if (active && j < 3) u[3 * v + j] = uo + (j == 0 ? a[0] : (j == 1 ? a[1] : a[2]));
}

// u_v += sum_i W_vi (x) e_i, entries batched four at a time.
__device__ __forceinline__ void prolong_sum(int k0, int k1, const int32_t* __restrict__ vh,
                                            const double* __restrict__ vw, const double* __restrict__ e,
                                            double& a0, double& a1, double& a2) {
  for (int kb = k0; kb < k1; kb += 4) {
    int h[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) h[u] = (kb + u < k1) ? vh[kb + u] : -1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (h[u] < 0) continue;
      const double* w = vw + 4 * int64_t(kb + u);
      const double* q = e + 12 * int64_t(h[u]);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        a0 += w[l] * q[l];
        a1 += w[l] * q[4 + l];
        a2 += w[l] * q[8 + l];
      }
    }
  }
}

// Stage 1: one thread per (v, j) entry of Z = H U.
template <typename HT>
__global__ void __launch_bounds__(256) k_galerkin_z(int64_t nz, int S, const int32_t* __restrict__ zptr,
                                                    const int32_t* __restrict__ zent, const HT* __restrict__ vals,
                                                    const double* __restrict__ vw, const uint8_t* __restrict__ zmask,
                                                    double* __restrict__ Z) {
  const int64_t z = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (z >= nz) return;
  double acc[36];
#pragma unroll
  for (int q = 0; q < 36; ++q) acc[q] = 0.0;
  if (!zmask[z]) {
    for (int e = zptr[z]; e < zptr[z + 1]; ++e) {
      const int64_t slot = zent[2 * e];
      const double* w = vw + 4 * int64_t(zent[2 * e + 1]);
      const HT* h = vals + vbase(slot, S);
      double hb[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) hb[q] = double(h[S * q]);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
          for (int l = 0; l < 4; ++l) acc[12 * a + 4 * b + l] += hb[3 * a + b] * w[l];
    }
  }
  double* out = Z + 36 * z;
#pragma unroll
  for (int q = 0; q < 36; ++q) out[q] = acc[q];
}

// Stage 2: one block per coarse pair (i <= j); entries staged through LDS.
__global__ void __launch_bounds__(256) k_galerkin_a(int r, const int32_t* __restrict__ pair_ij,
                                                    const int32_t* __restrict__ pptr,
                                                    const int32_t* __restrict__ pent, const double* __restrict__ vw,
                                                    const double* __restrict__ Z, double* __restrict__ A) {
  __shared__ double sw[64][4];
  __shared__ double sz[64][36];
  const int p = blockIdx.x;
  const int i = pair_ij[2 * p], j = pair_ij[2 * p + 1];
  const int t = threadIdx.x;
  // output (a,k),(b,l) handled by thread t < 144: a = t/48, k = (t/12)%4, b = (t%12)/4, l = t%4
  const int a = t / 48, k = (t / 12) % 4, b = (t % 12) / 4, l = t % 4;
  double acc = 0.0;
  for (int e0 = pptr[p]; e0 < pptr[p + 1]; e0 += 64) {
    const int ne = min(64, pptr[p + 1] - e0);
    __syncthreads();
    for (int q = t; q < ne * 40; q += blockDim.x) {
      const int e = q / 40, c = q % 40;
      const int kv = pent[2 * (e0 + e)], zz = pent[2 * (e0 + e) + 1];
      if (c < 4)
        sw[e][c] = vw[4 * int64_t(kv) + c];
      else
        sz[e][c - 4] = Z[36 * int64_t(zz) + (c - 4)];
    }
    __syncthreads();
    if (t < 144)
      for (int e = 0; e < ne; ++e) acc += sw[e][k] * sz[e][12 * a + 4 * b + l];
  }
  if (t < 144) {
    const int row = 12 * i + 4 * a + k, col = 12 * j + 4 * b + l;
    A[int64_t(row) * r + col] = acc;
    if (i != j) A[int64_t(col) * r + row] = acc;
  }
}

// Cubature stage 1 (Sec. 3.8): one thread per row of Z, written in the
// layout of k_galerkin_z so that k_galerkin_a forms U^T Z.  Element rows
// (tet t, local vertex a, handle j): Z = h^2 (w_t / V_t) sum_b H_t[a,b] (x) W_bj
// over the tet's unpinned vertices b carrying j; vertex rows (v, j):
// Z = (m_v I + h^2 (kappa b''(d_v) n n^T + D''_v)) (x) W_vj.
template <typename HT>
__global__ void __launch_bounds__(256) k_cub_z(int64_t nz, const int4* __restrict__ info,
                                               const double* __restrict__ scale, const int32_t* __restrict__ ent,
                                               const HT* __restrict__ He, const double* __restrict__ vw,
                                               const double* __restrict__ mass, const double* __restrict__ x,
                                               double h2, HalfSpace hs, double* __restrict__ Z) {
  const int64_t z = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (z >= nz) return;
  const int4 in = info[z];
  double acc[36];
#pragma unroll
  for (int q = 0; q < 36; ++q) acc[q] = 0.0;
  if (in.x >= 0) {
    const int a = in.y;
    for (int e = in.z; e < in.w; ++e) {
      const int b = ent[2 * e];
      const double* w = vw + 4 * int64_t(ent[2 * e + 1]);
      const int lo = min(a, b), hi = max(a, b);
      const HT* blk = He + 90 * int64_t(in.x) + 9 * (4 * lo - (lo * (lo - 1)) / 2 + (hi - lo));
      double hb[9];
      if (a <= b) {
#pragma unroll
        for (int q = 0; q < 9; ++q) hb[q] = double(blk[q]);
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) hb[3 * i + j] = double(blk[3 * j + i]);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int l = 0; l < 4; ++l) acc[12 * i + 4 * j + l] += hb[3 * i + j] * w[l];
    }
    const double sc = h2 * scale[z];
#pragma unroll
    for (int q = 0; q < 36; ++q) acc[q] *= sc;
  } else {
    const int64_t v = -1 - int64_t(in.x);
    double D[9];
    const double m = mass[v];
#pragma unroll
    for (int q = 0; q < 9; ++q) D[q] = (q % 4 == 0) ? m : 0.0;
    if (hs.on && m > 0.0) {
      const double y[3] = {x[3 * v], x[3 * v + 1], x[3 * v + 2]};
      double b, b1, b2;
      barrier_terms(hs.n[0] * y[0] + hs.n[1] * y[1] + hs.n[2] * y[2] - hs.off, hs.dhat, b, b1, b2);
      const double f = h2 * hs.kappa * b2;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) D[3 * i + j] += f * hs.n[i] * hs.n[j];
      if (hs.mu > 0.0) {
        double gf[3], Hf[9];
        friction_terms(hs, v, y, gf, Hf);
#pragma unroll
        for (int q = 0; q < 9; ++q) D[q] += h2 * Hf[q];
      }
    }
    const double* w = vw + 4 * int64_t(in.y);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int l = 0; l < 4; ++l) acc[12 * i + 4 * j + l] = D[3 * i + j] * w[l];
  }
  double* out = Z + 36 * z;
#pragma unroll
  for (int q = 0; q < 36; ++q) out[q] = acc[q];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static inline unsigned nblocks(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// Transfer operators of a basis: per-vertex weights W = phi [1, x - o]
// (prolongation), the transpose in handle order (vertices ascending) and the
// restriction chunks (handle i's entries in runs of at most kRChunk).
struct TransferLists {
  std::vector<int32_t> vptr, hptr, hv, hk;
  std::vector<double> vw, hw;
  std::vector<int4> chunk_info;
  std::vector<int2> hinfo;
};

static void transfer_lists(const ms_ctx* c, const Basis& B, TransferLists& T) {
  const int64_t n = c->n, nnz = B.vptr[n];
  const int m = B.m;
  T.vptr.assign(n + 1, 0);
  for (int64_t v = 0; v <= n; ++v) T.vptr[v] = int32_t(B.vptr[v]);
  T.vw.assign(4 * nnz, 0.0);
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = B.vptr[v]; k < B.vptr[v + 1]; ++k) {
      const int i = B.vhandle[k];
      T.vw[4 * k] = B.vphi[k];
      for (int d = 0; d < 3; ++d) T.vw[4 * k + 1 + d] = B.vphi[k] * (c->h_rest[3 * v + d] - B.origins[3 * i + d]);
    }
  T.hptr.assign(m + 1, 0);
  T.hv.assign(nnz, 0);
  T.hk.assign(nnz, 0);
  for (int64_t k = 0; k < nnz; ++k) T.hptr[B.vhandle[k] + 1]++;
  for (int i = 0; i < m; ++i) T.hptr[i + 1] += T.hptr[i];
  {
    std::vector<int32_t> fill(T.hptr.begin(), T.hptr.end() - 1);
    for (int64_t v = 0; v < n; ++v)
      for (int64_t k = B.vptr[v]; k < B.vptr[v + 1]; ++k) {
        const int32_t pos = fill[B.vhandle[k]]++;
        T.hv[pos] = int32_t(v);
        T.hk[pos] = int32_t(k);
      }
  }
  T.hw.assign(4 * size_t(std::max<int64_t>(nnz, 1)), 0.0);
  for (int64_t e = 0; e < nnz; ++e)
    for (int l = 0; l < 4; ++l) T.hw[4 * e + l] = T.vw[4 * size_t(T.hk[e]) + l];
  T.chunk_info.clear();
  T.hinfo.assign(m, make_int2(0, 0));
  for (int i = 0; i < m; ++i) {
    const int nchk = std::max(1, (T.hptr[i + 1] - T.hptr[i] + kRChunk - 1) / kRChunk);
    T.hinfo[i] = make_int2(int(T.chunk_info.size()), nchk);
    for (int q = 0; q < nchk; ++q) {
      const int e0 = T.hptr[i] + q * kRChunk;
      T.chunk_info.push_back(make_int4(i, e0, std::min(T.hptr[i + 1], e0 + kRChunk), 0));
    }
  }
}

// Installs only the transfer operators of B on c (prolongation rows,
// restriction chunks, coarse vector): the batched two-level preconditioner
// uses them on the union of the scenes' meshes while every scene keeps its
// own coarse matrix and inverse.  has_basis stays false on c.
ms_status install_transfer(ms_ctx* c, const Basis& B) {
  const int64_t n = c->n;
  if (B.m < 1 || int64_t(B.vptr.size()) != n + 1 || B.vptr[0] != 0 || B.vptr[n] < 1)
    return fail(c, MS_E_ARG, "bad transfer basis");
  TransferLists T;
  transfer_lists(c, B, T);
  Basis& D = c->basis;
  const int64_t nnz = B.vptr[n];
  const int32_t nrchunks = int32_t(T.chunk_info.size());
  ms_status s;
  if ((s = upload(c, &D.d_vptr, T.vptr.data(), T.vptr.size())) || (s = upload(c, &D.d_vh, B.vhandle.data(), nnz)) ||
      (s = upload(c, &D.d_vw, T.vw.data(), T.vw.size())) || (s = upload(c, &D.d_hv, T.hv.data(), nnz)) ||
      (s = upload(c, &D.d_hw, T.hw.data(), T.hw.size())) ||
      (s = upload(c, &D.d_chunk_info, T.chunk_info.data(), T.chunk_info.size())) ||
      (s = alloc_n(c, &D.d_rpart, 12 * size_t(nrchunks))) || (s = upload(c, &D.d_hinfo, T.hinfo.data(), T.hinfo.size())) ||
      (s = alloc_n(c, &c->d_e, 12 * size_t(B.m))))
    return s;
  D.nrchunks = nrchunks;
  D.m = B.m;
  D.nnz = nnz;
  c->r = 12 * B.m;
  return sync(c);
}

ms_status install_basis(ms_ctx* c, Basis&& B) {
  const int64_t n = c->n;
  const int m = B.m;
  if (m < 1) return fail(c, MS_E_ARG, "basis has no handles");
  if (int64_t(B.vptr.size()) != n + 1 || B.vptr[0] != 0) return fail(c, MS_E_ARG, "bad vptr");
  const int64_t nnz = B.vptr[n];
  if (nnz > (int64_t(1) << 30)) return fail(c, MS_E_ARG, "basis too large");
  if (nnz < 1) return fail(c, MS_E_ARG, "basis has no entries");
  B.nnz = nnz;
  for (int64_t k = 0; k < nnz; ++k)
    if (B.vhandle[k] < 0 || B.vhandle[k] >= m || !std::isfinite(B.vphi[k]))
      return fail(c, MS_E_ARG, "bad basis entry");
  TransferLists T;
  transfer_lists(c, B, T);
  std::vector<int32_t>& vptr = T.vptr;
  std::vector<double>& vw = T.vw;
  std::vector<int32_t>& hptr = T.hptr;
  std::vector<int32_t>& hv = T.hv;
  std::vector<int32_t>& hk = T.hk;
  std::vector<double>& hw = T.hw;
  std::vector<int4>& chunk_info = T.chunk_info;
  std::vector<int2>& hinfo = T.hinfo;
  const int32_t nrchunks = int32_t(chunk_info.size());
  // Galerkin stage-1 lists: for each vertex v the handles reachable through
  // its Hessian row, h'(v) = union of h(w) for w in N(v)
  const Pattern& P = c->pat;
  std::vector<int32_t> zvptr(n + 1, 0);
  std::vector<int32_t> zhandle;
  std::vector<int32_t> zptr(1, 0), zent;
  std::vector<uint8_t> zmask;
  std::vector<std::vector<std::pair<int, int>>> tmp;  // per handle in h'(v): (slot, k_w)
  std::vector<int> hpos(m, -1);
  std::vector<uint8_t> pinned(n, 0);
  for (int v : c->h_dbc) pinned[v] = 1;
  for (int64_t v = 0; v < n; ++v) {
    std::vector<int> hs;
    for (int32_t q = P.h_row_ptr[v]; q < P.h_row_ptr[v + 1]; ++q) {
      const int w = P.h_col[q];
      for (int64_t k = B.vptr[w]; k < B.vptr[w + 1]; ++k) hs.push_back(B.vhandle[k]);
    }
    std::sort(hs.begin(), hs.end());
    hs.erase(std::unique(hs.begin(), hs.end()), hs.end());
    tmp.assign(hs.size(), {});
    for (size_t a = 0; a < hs.size(); ++a) hpos[hs[a]] = int(a);
    for (int32_t q = P.h_row_ptr[v]; q < P.h_row_ptr[v + 1]; ++q) {
      const int w = P.h_col[q];
      if (pinned[w]) continue;  // U vanishes on eliminated DOFs
      const int64_t slot = P.h_slot_of_bsr[q];
      for (int64_t k = B.vptr[w]; k < B.vptr[w + 1]; ++k) tmp[hpos[B.vhandle[k]]].push_back({int(slot), int(k)});
    }
    for (size_t a = 0; a < hs.size(); ++a) {
      zhandle.push_back(hs[a]);
      for (auto& pr : tmp[a]) {
        zent.push_back(pr.first);
        zent.push_back(pr.second);
      }
      zptr.push_back(int32_t(zent.size() / 2));
      zmask.push_back(pinned[v] ? 1 : 0);
      hpos[hs[a]] = -1;
    }
    zvptr[v + 1] = int32_t(zhandle.size());
  }
  const int64_t nz = int64_t(zhandle.size());
  // stage-2 lists per coarse pair (i <= j): (k_v of (v,i), z index of (v,j))
  std::vector<std::vector<std::pair<int, int>>> pl;
  std::vector<std::pair<int, int>> pairs;
  {
    std::map<std::pair<int, int>, int> pid;
    std::vector<std::vector<std::pair<int, int>>> lists;
    for (int64_t v = 0; v < n; ++v) {
      if (pinned[v]) continue;
      for (int64_t k = B.vptr[v]; k < B.vptr[v + 1]; ++k) {
        const int i = B.vhandle[k];
        for (int32_t z = zvptr[v]; z < zvptr[v + 1]; ++z) {
          const int j = zhandle[z];
          if (j < i) continue;
          auto key = std::make_pair(i, j);
          auto it = pid.find(key);
          int id;
          if (it == pid.end()) {
            id = int(lists.size());
            pid[key] = id;
            lists.emplace_back();
          } else {
            id = it->second;
          }
          lists[id].push_back({int(k), int(z)});
        }
      }
    }
    for (auto& kv : pid) {
      pairs.push_back(kv.first);
      pl.push_back(std::move(lists[kv.second]));
    }
  }
  std::vector<int32_t> pair_ij, pptr(1, 0), pent;
  for (size_t p = 0; p < pairs.size(); ++p) {
    pair_ij.push_back(pairs[p].first);
    pair_ij.push_back(pairs[p].second);
    for (auto& e : pl[p]) {
      pent.push_back(e.first);
      pent.push_back(e.second);
    }
    pptr.push_back(int32_t(pent.size() / 2));
  }
  // paper mode: the affine origin (rest centre of mass) and the refinement
  // iteration count from the partitions' hop diameters (Sec. 3.7.2: the mean
  // over partitions of the largest number of edge hops, over mesh edges
  // joining two of the partition's vertices, from the vertex nearest the
  // handle origin; 20 when that mean is at most 30, else 40)
  {
    double msum = 0.0, o[3] = {0, 0, 0};
    for (int64_t v = 0; v < n; ++v) {
      msum += c->h_mass[v];
      for (int d = 0; d < 3; ++d) o[d] += c->h_mass[v] * c->h_rest[3 * v + d];
    }
    for (int d = 0; d < 3; ++d) c->oa[d] = msum > 0 ? o[d] / msum : 0.0;
  }
  c->refine_auto = 20;
  if (int64_t(B.part.size()) == c->T && !B.part.empty() && B.part[0] >= 0) {
    std::vector<std::vector<int32_t>> pverts(m);
    {
      std::vector<int32_t> last(n, -1);
      for (int64_t t = 0; t < c->T; ++t) {
        const int l = B.part[t];
        if (l < 0 || l >= m) continue;
        for (int q = 0; q < 4; ++q) {
          const int32_t v = c->h_tets[4 * t + q];
          if (last[v] != l) {
            pverts[l].push_back(v);
            last[v] = l;
          }
        }
      }
    }
    std::vector<int32_t> mark(n, -1), dist(n, 0), queue;
    double hop_sum = 0.0;
    int counted = 0;
    for (int l = 0; l < m; ++l) {
      auto& pv = pverts[l];
      std::sort(pv.begin(), pv.end());
      pv.erase(std::unique(pv.begin(), pv.end()), pv.end());
      if (pv.empty()) continue;
      int32_t start = pv[0];
      double best = 1e300;
      for (int32_t v : pv) {
        double dd = 0.0;
        for (int d = 0; d < 3; ++d) dd += (c->h_rest[3 * v + d] - B.origins[3 * l + d]) * (c->h_rest[3 * v + d] - B.origins[3 * l + d]);
        if (dd < best) best = dd, start = v;
      }
      for (int32_t v : pv) mark[v] = l;
      queue.assign(1, start);
      dist[start] = 0;
      mark[start] = -2 - l;
      int far = 0;
      for (size_t qh = 0; qh < queue.size(); ++qh) {
        const int32_t v = queue[qh];
        far = std::max(far, dist[v]);
        for (int32_t k = c->pat.h_row_ptr[v]; k < c->pat.h_row_ptr[v + 1]; ++k) {
          const int32_t w = c->pat.h_col[k];
          if (mark[w] == l) {
            mark[w] = -2 - l;
            dist[w] = dist[v] + 1;
            queue.push_back(w);
          }
        }
      }
      hop_sum += far;
      ++counted;
    }
    if (counted > 0) c->refine_auto = (hop_sum / counted) <= 30.0 ? 20 : 40;
  }
  // coarse mass matrix (U^T M U) and its inverse for the coarse coordinates
  const int r = 12 * m;
  const int rp = coarse_pad(r);
  std::vector<double> G(size_t(4 * m) * 4 * m, 0.0);  // sum_v m_v W_vi W_vj^T  [(i,k),(j,l)]
  for (int64_t v = 0; v < n; ++v)
    for (int64_t a = B.vptr[v]; a < B.vptr[v + 1]; ++a)
      for (int64_t b = B.vptr[v]; b < B.vptr[v + 1]; ++b)
        for (int k = 0; k < 4; ++k)
          for (int l = 0; l < 4; ++l)
            G[size_t(4 * B.vhandle[a] + k) * (4 * m) + 4 * B.vhandle[b] + l] += c->h_mass[v] * vw[4 * a + k] * vw[4 * b + l];
  // invert G (SPD up to null directions) by Cholesky with pivot regularisation
  const int g = 4 * m;
  std::vector<double> Lg(G);
  double gmax = 0.0;
  for (int i = 0; i < g; ++i) gmax = std::max(gmax, G[size_t(i) * g + i]);
  for (int k = 0; k < g; ++k) {
    double d = Lg[size_t(k) * g + k];
    for (int q = 0; q < k; ++q) d -= Lg[size_t(k) * g + q] * Lg[size_t(k) * g + q];
    if (!(d > 1e-13 * gmax)) d = std::max(gmax, 1e-300);
    d = std::sqrt(d);
    Lg[size_t(k) * g + k] = d;
    for (int i = k + 1; i < g; ++i) {
      double s = Lg[size_t(i) * g + k];
      for (int q = 0; q < k; ++q) s -= Lg[size_t(i) * g + q] * Lg[size_t(k) * g + q];
      Lg[size_t(i) * g + k] = s / d;
    }
  }
  std::vector<double> Ginv(size_t(g) * g, 0.0);
  for (int col = 0; col < g; ++col) {
    std::vector<double> y(g, 0.0);
    for (int i = 0; i < g; ++i) {
      double s = (i == col) ? 1.0 : 0.0;
      for (int q = 0; q < i; ++q) s -= Lg[size_t(i) * g + q] * y[q];
      y[i] = s / Lg[size_t(i) * g + i];
    }
    for (int i = g - 1; i >= 0; --i) {
      double s = y[i];
      for (int q = i + 1; q < g; ++q) s -= Lg[size_t(q) * g + i] * y[q];
      y[i] = s / Lg[size_t(i) * g + i];
    }
    for (int i = 0; i < g; ++i) Ginv[size_t(i) * g + col] = y[i];
  }
  // expand to the r x r inverse of U^T M U = G (x) I_3 in (handle, a, k) order
  std::vector<double> Minv(size_t(r) * r, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 4; ++k)
          for (int l = 0; l < 4; ++l)
            Minv[size_t(12 * i + 4 * a + k) * r + 12 * j + 4 * a + l] = Ginv[size_t(4 * i + k) * g + 4 * j + l];
  // upload
  Basis& D = c->basis;
  ms_status s;
  if ((s = upload(c, &D.d_vptr, vptr.data(), vptr.size())) || (s = upload(c, &D.d_vh, B.vhandle.data(), nnz)) ||
      (s = upload(c, &D.d_vw, vw.data(), vw.size())) || (s = upload(c, &D.d_hptr, hptr.data(), hptr.size())) ||
      (s = upload(c, &D.d_hv, hv.data(), nnz)) || (s = upload(c, &D.d_hk, hk.data(), nnz)) ||
      (s = upload(c, &D.d_zptr, zptr.data(), zptr.size())) || (s = upload(c, &D.d_zent, zent.data(), zent.size())) ||
      (s = upload(c, &D.d_zmask, zmask.data(), zmask.size())) || (s = alloc_n(c, &D.d_Z, 36 * std::max<int64_t>(nz, 1))) ||
      (s = upload(c, &D.d_pair_ij, pair_ij.data(), pair_ij.size())) ||
      (s = upload(c, &D.d_pair_ptr, pptr.data(), pptr.size())) ||
      (s = upload(c, &D.d_pair_ent, pent.data(), pent.size())) ||
      (s = upload(c, &D.d_Minv, Minv.data(), Minv.size())) || (s = alloc_n(c, &c->d_c, r)) ||
      (s = upload(c, &D.d_hw, hw.data(), hw.size())) ||
      (s = upload(c, &D.d_chunk_info, chunk_info.data(), chunk_info.size())) ||
      (s = alloc_n(c, &D.d_rpart, 12 * size_t(nrchunks))) || (s = upload(c, &D.d_hinfo, hinfo.data(), hinfo.size())) ||
      (s = alloc_n(c, &c->d_Ainv32, size_t(rp) * rp)) ||
      (s = alloc_n(c, &c->d_e, r)) || (s = alloc_n(c, &c->d_Ac, size_t(r) * r)) ||
      (s = alloc_n(c, &c->d_Lc, size_t(rp) * rp)) || (s = alloc_n(c, &c->d_Ainv, size_t(rp) * rp)) ||
      (s = alloc_n(c, &c->d_Y, size_t(rp) * rp)) || (s = alloc_n(c, &c->d_Ldiag, size_t(rp) * 64)) ||
      (s = alloc_n(c, &c->d_Linvd, size_t(rp) * 64)) || (s = alloc_n(c, &c->d_diag0, rp + 1)) || (s = alloc_n(c, &c->d_nreg, 4)))
    return s;
  D.nrchunks = nrchunks;
  D.m = m;
  D.nnz = nnz;
  D.nz = nz;
  D.npairs = int32_t(pairs.size());
  D.pair_L = int64_t(pent.size() / 2);
  D.z_L = int64_t(zent.size() / 2);
  D.origins = std::move(B.origins);
  D.vptr = std::move(B.vptr);
  D.vhandle = std::move(B.vhandle);
  D.vphi = std::move(B.vphi);
  D.part = std::move(B.part);
  c->r = r;
  c->rp = rp;
  c->has_basis = true;
  c->coarse_valid = 0;
  c->cub.built = false;
  for (auto& row : c->cg_graph)
    for (int pc = 1; pc < 4; ++pc)
      if (row[pc]) {
        (void)hipGraphExecDestroy(row[pc]);
        row[pc] = nullptr;
      }
  return sync(c);
}

// Coarse matrix with the elastic part integrated by the installed cubature.
static ms_status launch_galerkin_cubature(ms_ctx* c, int prec, const double* x, double h2) {
  Cubature& C = c->cub;
  if (!C.present) return fail(c, MS_E_ORDER, "no cubature installed");
  if (!C.built) {
    ms_status s = build_cubature_lists(c);
    if (s) return s;
  }
  MS_HIP(hipMemsetAsync(c->d_Ac, 0, size_t(c->r) * c->r * sizeof(double), c->stream));
  if (C.nz > 0) {
    if (prec == MS_PREC_FP64)
      k_cub_z<double><<<nblocks(C.nz, 256), 256, 0, c->stream>>>(C.nz, C.d_info, C.d_scale, C.d_ent, c->d_He,
                                                                 c->basis.d_vw, c->d_mass, x, h2, hs_of(c), C.d_Z);
    else
      k_cub_z<float><<<nblocks(C.nz, 256), 256, 0, c->stream>>>(C.nz, C.d_info, C.d_scale, C.d_ent, c->d_He32,
                                                                c->basis.d_vw, c->d_mass, x, h2, hs_of(c), C.d_Z);
  }
  if (C.npairs > 0)
    k_galerkin_a<<<unsigned(C.npairs), 256, 0, c->stream>>>(c->r, C.d_pair_ij, C.d_pair_ptr, C.d_pair_ent,
                                                           c->basis.d_vw, C.d_Z, c->d_Ac);
  return MS_OK;
}

// Average duration of the coarse-matrix integration (exact Galerkin or
// cubature, whichever is selected) on the last assembled Hessian, over reps
// back-to-back launches bracketed by events on the library stream.
ms_status time_coarse_matrix(ms_ctx* c, int prec, int reps, double* avg_us, double* bytes) {
  if (!c->has_basis) return fail(c, MS_E_ORDER, "no basis");
  if (reps < 1) return fail(c, MS_E_ARG, "the coarse matrix is timed by replays (reps >= 1)");
  if (!c->asm_x) return fail(c, MS_E_ORDER, "nothing assembled yet");
  ms_status s = launch_galerkin(c, prec, c->asm_x, c->asm_h2);  // builds the cubature lists if needed
  if (s) return s;
  hipEvent_t e0, e1;
  MS_HIP(hipEventCreate(&e0));
  MS_HIP(hipEventCreate(&e1));
  MS_HIP(hipEventRecord(e0, c->stream));
  for (int k = 0; k < reps && !s; ++k) s = launch_galerkin(c, prec, c->asm_x, c->asm_h2);
  MS_HIP(hipEventRecord(e1, c->stream));
  MS_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  MS_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s) return s;
  *avg_us = 1e3 * double(ms) / reps;
  *bytes = 0.0;
  c->coarse_valid = 0;  // the factor no longer matches a freshly integrated matrix
  return MS_OK;
}

ms_status launch_galerkin(ms_ctx* c, int prec, const double* x, double h2) {
  if (!c->has_basis) return fail(c, MS_E_ORDER, "no basis");
  if (c->coarse_mode == MS_COARSE_CUBATURE) return launch_galerkin_cubature(c, prec, x, h2);
  Basis& D = c->basis;
  MS_HIP(hipMemsetAsync(c->d_Ac, 0, size_t(c->r) * c->r * sizeof(double), c->stream));
  if (D.nz > 0) {
    if (prec == MS_PREC_FP64)
      k_galerkin_z<double><<<nblocks(D.nz, 256), 256, 0, c->stream>>>(D.nz, c->pat.S, D.d_zptr, D.d_zent, c->d_vals, D.d_vw,
                                                                      D.d_zmask, D.d_Z);
    else
      k_galerkin_z<float><<<nblocks(D.nz, 256), 256, 0, c->stream>>>(D.nz, c->pat.S, D.d_zptr, D.d_zent, c->d_vals32, D.d_vw,
                                                                     D.d_zmask, D.d_Z);
  }
  if (D.npairs > 0)
    k_galerkin_a<<<unsigned(D.npairs), 256, 0, c->stream>>>(c->r, D.d_pair_ij, D.d_pair_ptr, D.d_pair_ent, D.d_vw,
                                                           D.d_Z, c->d_Ac);
  return MS_OK;
}

// e = A^-1 c with the FP32 inverse in mixed-precision steps (also in their
// FP64 iterations), else the FP64 inverse.
void launch_coarse_gemv(ms_ctx* c, int prec, const double* scal) {
  Basis& D = c->basis;
  const unsigned nb = nblocks(c->r, kGemvRows);
  const size_t lds = size_t(c->r) * sizeof(double);
  const int direct = (D.nrchunks == D.m && c->r <= kGemvPart * 64 * kGemvRows) ? 1 : 0;
  if (prec == MS_PREC_MIXED || c->coarse_f32)
    k_coarse_gemv<float><<<nb, 64 * kGemvRows, lds, c->stream>>>(c->r, c->rp, c->d_Ainv32, D.d_hinfo, D.d_rpart,
                                                                 c->d_e, scal, direct);
  else
    k_coarse_gemv<double><<<nb, 64 * kGemvRows, lds, c->stream>>>(c->r, c->rp, c->d_Ainv, D.d_hinfo, D.d_rpart,
                                                                  c->d_e, scal, direct);
}

void launch_prolong_add(ms_ctx* c, double* target, const double* scal) {
  Basis& D = c->basis;
  k_prolong8<<<nblocks(8 * c->n, 256), 256, 0, c->stream>>>(c->n, D.d_vptr, D.d_vh, D.d_vw, c->d_e, c->d_pinned,
                                                             target, scal);
}

// Restriction partials of U^T (weight .* v) into d_rpart.
void launch_restrict(ms_ctx* c, const double* v, const double* weight, const double* scal) {
  Basis& D = c->basis;
  k_restrict<<<unsigned(D.nrchunks), kRThreads, 0, c->stream>>>(D.d_chunk_info, D.d_hv, D.d_hw, v, weight, D.d_rpart,
                                                          scal);
}

// u += U A^-1 U^T v with v = r (from_w false) or the scratch vector w.
void launch_coarse_correction(ms_ctx* c, int prec, bool from_w) {
  launch_restrict(c, from_w ? c->d_w : c->d_r, nullptr, c->d_scal);
  launch_coarse_gemv(c, prec, c->d_scal);
  launch_prolong_add(c, c->d_u, c->d_scal);
}

// Preconditioner applied to r, with u = S r already in place.
void launch_precond_apply(ms_ctx* c, int prec, int pc) {
  if (pc == MS_PC_TWO_LEVEL_ADDITIVE) {
    launch_coarse_correction(c, prec, false);
  } else if (pc == MS_PC_TWO_LEVEL) {
    launch_spmv_resid(c, prec, false);  // w = r - H u
    launch_coarse_correction(c, prec, true);
  } else if (pc == MS_PC_TWO_LEVEL_VCYCLE) {  // u = L r on entry
    launch_spmv_resid(c, prec, false);        // w = r - H u
    launch_coarse_correction(c, prec, true);  // u += Q w
    launch_spmv_resid(c, prec, false);        // w = r - H u
    launch_bj_add(c, prec);                   // u += L w
  }
}

// d = U e with e already computed (coarse start of PCG).
__global__ void __launch_bounds__(64) k_prolong_set(int64_t n, const int32_t* __restrict__ vptr,
                                                     const int32_t* __restrict__ vh, const double* __restrict__ vw,
                                                     const double* __restrict__ e, const uint8_t* __restrict__ pinned,
                                                     double* __restrict__ d, const double* __restrict__ scal) {
  if (scal && scal[S_DONE] != 0.0) return;
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (!(pinned && pinned[v])) prolong_sum(vptr[v], vptr[v + 1], vh, vw, e, a0, a1, a2);
  d[3 * v] = a0;
  d[3 * v + 1] = a1;
  d[3 * v + 2] = a2;
}

void launch_prolong_set_d(ms_ctx* c) {
  Basis& D = c->basis;
  k_prolong_set<<<nblocks(c->n, 64), 64, 0, c->stream>>>(c->n, D.d_vptr, D.d_vh, D.d_vw, c->d_e, c->d_pinned,
                                                           c->d_d, c->d_scal);
}

// PCG starting vector d_0 = Q r_0 (r_0 = -g): afterwards r = -g - H d_0 and
// u = S r.
void launch_coarse_start(ms_ctx* c, int prec) {
  launch_restrict(c, c->d_r, nullptr, c->d_scal);
  launch_coarse_gemv(c, prec, c->d_scal);
  launch_prolong_set_d(c);
  launch_spmv_resid(c, prec, true);  // r = r - H d
  launch_bj(c, prec);                 // u = S r
}

// q = (U^T M U)^-1 U^T M (x - x_rest), on the device; result copied to host.
ms_status coarse_coordinates(ms_ctx* c, const double* x_dev, double* q_host, double* q_dev) {
  Basis& D = c->basis;
  // d_w <- x - rest (scratch)
  k_sub<<<nblocks(3 * c->n, 256), 256, 0, c->stream>>>(3 * c->n, x_dev, c->d_rest, c->d_w);
  launch_restrict(c, c->d_w, c->d_mass, nullptr);
  k_coarse_gemv<double><<<nblocks(c->r, kGemvRows), 64 * kGemvRows, size_t(c->r) * sizeof(double), c->stream>>>(
      c->r, c->r, D.d_Minv, D.d_hinfo, D.d_rpart, q_dev ? q_dev : c->d_e, nullptr, 0);
  if (q_host)
    MS_HIP(hipMemcpyAsync(q_host, q_dev ? q_dev : c->d_e, c->r * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

}  // namespace ms

using namespace ms;

extern "C" {

ms_status ms_build_basis(ms_ctx* c, const ms_basis_params* p) {
  if (!c) return MS_E_ARG;
  if (c->stage < 2) return fail(c, MS_E_ORDER, "upload mesh and material first");
  ms_basis_params P;
  if (p)
    P = *p;
  else
    ms_basis_defaults(&P);
  if (P.n_handles < 1 || P.n_handles > c->n) return fail(c, MS_E_ARG, "n_handles out of range");
  Basis B;
  const auto t0 = std::chrono::steady_clock::now();
  c->basis_gpu_min = std::max(0, P.gpu_min_unknowns);
  ms_status s = build_basis_host(c, P, B);
  c->basis_gpu_min = 0;
  c->basis_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (s) return s;
  return install_basis(c, std::move(B));
}

ms_status ms_get_basis_stats(const ms_ctx* c, int32_t* gpu_solves, double* seconds) {
  if (!c) return MS_E_ARG;
  if (gpu_solves) *gpu_solves = c->basis_gpu_solves;
  if (seconds) *seconds = c->basis_seconds;
  return MS_OK;
}

ms_status ms_set_basis(ms_ctx* c, int32_t m, const double* origins, const int64_t* vptr, const int32_t* vhandle,
                       const double* vphi) {
  if (!c || !origins || !vptr || !vhandle || !vphi || m < 1) return MS_E_ARG;
  if (c->stage < 2) return fail(c, MS_E_ORDER, "upload mesh and material first");
  Basis B;
  B.m = m;
  B.origins.assign(origins, origins + 3 * m);
  B.vptr.assign(vptr, vptr + c->n + 1);
  const int64_t nnz = B.vptr[c->n];
  if (nnz < 0) return fail(c, MS_E_ARG, "bad vptr");
  for (int64_t v = 0; v < c->n; ++v)
    if (B.vptr[v + 1] < B.vptr[v]) return fail(c, MS_E_ARG, "vptr not monotone");
  B.vhandle.assign(vhandle, vhandle + nnz);
  B.vphi.assign(vphi, vphi + nnz);
  B.part.assign(c->T, -1);
  return install_basis(c, std::move(B));
}

ms_status ms_get_basis_size(const ms_ctx* c, int32_t* m, int64_t* nnz) {
  if (!c || !m || !nnz) return MS_E_ARG;
  if (!c->has_basis) return fail(const_cast<ms_ctx*>(c), MS_E_ORDER, "no basis");
  *m = c->basis.m;
  *nnz = c->basis.nnz;
  return MS_OK;
}

ms_status ms_get_basis(const ms_ctx* c, double* origins, int64_t* vptr, int32_t* vhandle, double* vphi,
                       int32_t* part) {
  if (!c) return MS_E_ARG;
  if (!c->has_basis) return fail(const_cast<ms_ctx*>(c), MS_E_ORDER, "no basis");
  const Basis& B = c->basis;
  if (origins) std::memcpy(origins, B.origins.data(), B.origins.size() * sizeof(double));
  if (vptr) std::memcpy(vptr, B.vptr.data(), B.vptr.size() * sizeof(int64_t));
  if (vhandle) std::memcpy(vhandle, B.vhandle.data(), B.vhandle.size() * sizeof(int32_t));
  if (vphi) std::memcpy(vphi, B.vphi.data(), B.vphi.size() * sizeof(double));
  if (part) {
    if (B.part.empty())
      std::fill(part, part + c->T, -1);
    else
      std::memcpy(part, B.part.data(), B.part.size() * sizeof(int32_t));
  }
  return MS_OK;
}

ms_status ms_get_coarse_matrix(ms_ctx* c, double* A) {
  if (!c || !A) return MS_E_ARG;
  if (!c->has_basis || !c->eval_valid) return fail(c, MS_E_ORDER, "needs a basis and ms_eval");
  MS_HIP(hipMemcpyAsync(A, c->d_Ac, size_t(c->r) * c->r * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

ms_status ms_get_coarse(ms_ctx* c, double* q) {
  if (!c || !q) return MS_E_ARG;
  if (!c->has_basis) return fail(c, MS_E_ORDER, "no basis");
  if (c->stage < 3) return fail(c, MS_E_ORDER, "no state");
  return coarse_coordinates(c, c->d_x, q, nullptr);
}

}  // extern "C"
