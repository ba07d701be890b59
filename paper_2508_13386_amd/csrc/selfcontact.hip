// Continuous collision detection of surface primitive pairs for IPC
// self-contact (the paper filters every search direction with additive CCD;
// Sec. 3.9 line search, Sec. 4): one thread per point-triangle or
// edge-edge pair, distance evaluations only.
//
// Additive CCD (Li et al., "Codimensional Incremental Potential Contact",
// 2021) with zero thickness: the mean displacement of the pair is removed,
// l_p bounds the remaining relative speed (point: |p_0| + max_i |p_i| over
// the triangle; edges: max over each edge's endpoints, summed), and the
// pair advances in steps that cannot close more than 90% of the current
// gap (the first one (1 - s) of it).  The pair is reported hit once the gap
// falls below s times the initial gap; the returned time is the last one
// before that step, at which the gap was still at least s d_0.  Reaching
// t_max first reports no hit; an iteration cap reports a hit at the time
// reached (still conservative).
//
// Broad and narrow phase of the constraint set: every surface primitive's
// box, inflated by d_hat / 2, is entered into each grid cell it overlaps
// (cells keyed by their integer coordinates, no hashing collisions); the
// entries are sorted by cell; vertex-triangle and edge-edge pairs sharing a
// cell become candidates (duplicates from several shared cells removed by
// sorting and uniquing the pair keys); candidates closer than d_hat by the
// exact distance are kept, in ascending key order.  Counts go through
// prefix sums, never atomics, so the output is deterministic.
#include <algorithm>
#include <array>
#include <cmath>
#include <iterator>
#include <string>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include "contact.h"
#include "ms_internal.h"

namespace ms {
namespace {

__device__ __forceinline__ double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void sub3(const double* a, const double* b, double* c) {
  c[0] = a[0] - b[0];
  c[1] = a[1] - b[1];
  c[2] = a[2] - b[2];
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// squared distance from p to the closed segment [a, b]
__device__ double seg_d2(const double* p, const double* a, const double* b) {
  double ab[3], ap[3];
  sub3(b, a, ab);
  sub3(p, a, ap);
  const double t = fmin(fmax(dot3(ap, ab) / dot3(ab, ab), 0.0), 1.0);
  double r[3];
  for (int i = 0; i < 3; ++i) r[i] = p[i] - (a[i] + t * ab[i]);
  return dot3(r, r);
}

// point x[0..3) to the closed triangle x[3..12): the plane distance when the
// projection falls inside, else the nearest edge
__device__ double pt_d2(const double* x) {
  const double *p = x, *t0 = x + 3, *t1 = x + 6, *t2 = x + 9;
  double e0[3], e1[3], w[3], n[3];
  sub3(t1, t0, e0);
  sub3(t2, t0, e1);
  sub3(p, t0, w);
  cross3(e0, e1, n);
  const double d00 = dot3(e0, e0), d01 = dot3(e0, e1), d11 = dot3(e1, e1);
  const double d20 = dot3(w, e0), d21 = dot3(w, e1);
  const double den = d00 * d11 - d01 * d01;
  const double v = (d11 * d20 - d01 * d21) / den;
  const double u = (d00 * d21 - d01 * d20) / den;
  if (v >= 0.0 && u >= 0.0 && u + v <= 1.0) {
    const double h = dot3(w, n);
    return h * h / dot3(n, n);
  }
  return fmin(fmin(seg_d2(p, t0, t1), seg_d2(p, t1, t2)), seg_d2(p, t0, t2));
}

// closed segments [x0, x1] and [x2, x3]: the line distance when both closest
// parameters are interior, else the nearest endpoint-to-segment distance
__device__ double ee_d2(const double* x) {
  const double *a0 = x, *a1 = x + 3, *b0 = x + 6, *b1 = x + 9;
  double u[3], v[3], w[3];
  sub3(a1, a0, u);
  sub3(b1, b0, v);
  sub3(a0, b0, w);
  const double uu = dot3(u, u), uv = dot3(u, v), vv = dot3(v, v), uw = dot3(u, w), vw = dot3(v, w);
  const double den = uu * vv - uv * uv;
  if (den > 1e-12 * uu * vv) {
    const double s = (uv * vw - vv * uw) / den;
    const double t = (uu * vw - uv * uw) / den;
    if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
      double n[3];
      cross3(u, v, n);
      const double h = dot3(w, n);
      return h * h / dot3(n, n);
    }
  }
  return fmin(fmin(seg_d2(a0, b0, b1), seg_d2(a1, b0, b1)), fmin(seg_d2(b0, a0, a1), seg_d2(b1, a0, a1)));
}

__global__ void __launch_bounds__(256) k_accd(int64_t np, const int32_t* __restrict__ kind,
                                              const double* __restrict__ x12, const double* __restrict__ p12,
                                              double s, double t_max, int max_iter, double* __restrict__ toi,
                                              int32_t* __restrict__ hit) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= np) return;
  double x[12], p[12];
  for (int k = 0; k < 12; ++k) {
    x[k] = x12[12 * q + k];
    p[k] = p12[12 * q + k];
  }
  const bool pt = kind[q] == 0;
  double mean[3];
  for (int i = 0; i < 3; ++i) mean[i] = (p[i] + p[3 + i] + p[6 + i] + p[9 + i]) / 4.0;
  double nrm[4];
  for (int a = 0; a < 4; ++a) {
    for (int i = 0; i < 3; ++i) p[3 * a + i] -= mean[i];
    nrm[a] = sqrt(dot3(p + 3 * a, p + 3 * a));
  }
  const double lp = pt ? nrm[0] + fmax(fmax(nrm[1], nrm[2]), nrm[3]) : fmax(nrm[0], nrm[1]) + fmax(nrm[2], nrm[3]);
  if (lp == 0.0) {
    hit[q] = 0;
    toi[q] = t_max;
    return;
  }
  double d = sqrt(pt ? pt_d2(x) : ee_d2(x));
  const double g = s * d;
  double t = 0.0;
  double tl = (1.0 - s) * d / lp;
  for (int it = 0; it < max_iter; ++it) {
    for (int k = 0; k < 12; ++k) x[k] += tl * p[k];
    d = sqrt(pt ? pt_d2(x) : ee_d2(x));
    if (t > 0.0 && d < g) break;
    t += tl;
    if (t > t_max) {
      hit[q] = 0;
      toi[q] = t_max;
      return;
    }
    tl = 0.9 * d / lp;
  }
  hit[q] = 1;
  toi[q] = t;
}

constexpr int64_t kCellBias = int64_t(1) << 20;  // cell coordinates in (-2^20, 2^20)

__device__ __forceinline__ int64_t cell_key(int64_t ix, int64_t iy, int64_t iz) {
  return ((ix + kCellBias) << 42) | ((iy + kCellBias) << 21) | (iz + kCellBias);
}

// box of primitive q (k vertices), inflated by r, in cell coordinates; with
// x2 the box spans both positions (the swept box of a linear motion)
__device__ __forceinline__ void prim_cells(const double* __restrict__ x, const double* __restrict__ x2,
                                           const int32_t* __restrict__ vid, int k, double r, double inv_cell,
                                           int64_t lo[3], int64_t hi[3]) {
  for (int i = 0; i < 3; ++i) {
    double a = x[3 * int64_t(vid[0]) + i], b = a;
    for (int j = 0; j < k; ++j) {
      const double v = x[3 * int64_t(vid[j]) + i];
      a = fmin(a, v);
      b = fmax(b, v);
      if (x2) {
        const double w = x2[3 * int64_t(vid[j]) + i];
        a = fmin(a, w);
        b = fmax(b, w);
      }
    }
    lo[i] = int64_t(floor((a - r) * inv_cell));
    hi[i] = int64_t(floor((b + r) * inv_cell));
  }
}

// Entries of primitives [0, np): primitive q has k vertices prims[k q ..].
// Pass 0 counts the cells of each primitive into cnt; pass 1 writes (cell,
// tag + id) from off[q] on, id the vertex id for vertices (k = 1) and q
// otherwise.
__global__ void __launch_bounds__(256) k_cells(int64_t np, const int32_t* __restrict__ prims, int k,
                                               const double* __restrict__ x, const double* __restrict__ x2,
                                               double r, double inv_cell, int64_t tag, int pass,
                                               int64_t* __restrict__ cnt, const int64_t* __restrict__ off,
                                               int64_t* __restrict__ keys, int64_t* __restrict__ vals) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= np) return;
  int64_t lo[3], hi[3];
  prim_cells(x, x2, prims + int64_t(k) * q, k, r, inv_cell, lo, hi);
  if (pass == 0) {
    cnt[q] = (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
    return;
  }
  int64_t o = off[q];
  const int64_t id = k == 1 ? int64_t(prims[q]) : q;  // vertices by vertex id, others by index
  for (int64_t ix = lo[0]; ix <= hi[0]; ++ix)
    for (int64_t iy = lo[1]; iy <= hi[1]; ++iy)
      for (int64_t iz = lo[2]; iz <= hi[2]; ++iz) {
        keys[o] = cell_key(ix, iy, iz);
        vals[o] = tag + id;
        ++o;
      }
}

// cell_end[e] = one past the last entry of entry e's cell (sorted keys)
__global__ void __launch_bounds__(256) k_cell_end(int64_t ne, const int64_t* __restrict__ keys,
                                                  int64_t* __restrict__ cell_end) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int64_t f = e + 1;
  while (f < ne && keys[f] == keys[e]) ++f;
  cell_end[e] = f;
}

constexpr int64_t kTri = int64_t(1) << 40;  // value tag of triangle entries

// Candidate pairs sharing a cell.  Vertex-triangle: a vertex entry against
// the triangle entries of its cell (the vertex not in the triangle), key
// v << 32 | t.  Edge-edge: an edge entry against the later entries of its
// cell (no shared vertex), key min << 32 | max.  Pass 0 counts, pass 1
// writes at off[e].
__global__ void __launch_bounds__(256) k_candidates(int64_t ne, const int64_t* __restrict__ keys,
                                                    const int64_t* __restrict__ vals,
                                                    const int64_t* __restrict__ cell_end, int ee,
                                                    const int32_t* __restrict__ tris,
                                                    const int32_t* __restrict__ edges, int pass,
                                                    int64_t* __restrict__ cnt, const int64_t* __restrict__ off,
                                                    int64_t* __restrict__ out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int64_t end = cell_end[e];
  int64_t c = 0;
  int64_t o = pass ? off[e] : 0;
  if (!ee) {
    if (vals[e] >= kTri) {
      if (pass == 0) cnt[e] = 0;
      return;
    }
    const int64_t v = vals[e];
    int64_t f = e;  // the cell starts at or before e: scan back to its first entry
    while (f > 0 && keys[f - 1] == keys[e]) --f;
    for (; f < end; ++f) {
      if (vals[f] < kTri) continue;
      const int64_t t = vals[f] - kTri;
      const int32_t* tv = tris + 3 * t;
      if (tv[0] == v || tv[1] == v || tv[2] == v) continue;
      if (pass) out[o++] = (v << 32) | t;
      ++c;
    }
  } else {
    const int64_t a = vals[e];
    const int32_t* av = edges + 2 * a;
    for (int64_t f = e + 1; f < end; ++f) {
      const int64_t b = vals[f];
      if (b == a) continue;
      const int32_t* bv = edges + 2 * b;
      if (av[0] == bv[0] || av[0] == bv[1] || av[1] == bv[0] || av[1] == bv[1]) continue;
      if (pass) out[o++] = (min(a, b) << 32) | max(a, b);
      ++c;
    }
  }
  if (pass == 0) cnt[e] = c;
}

// exact narrow phase of unique candidates: keep[c] = 1 when closer than d_hat
__global__ void __launch_bounds__(256) k_narrow(int64_t nc, const int64_t* __restrict__ cand, int ee,
                                                const double* __restrict__ x, const int32_t* __restrict__ tris,
                                                const int32_t* __restrict__ edges, double dhat2,
                                                int64_t* __restrict__ keep) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int64_t hi = cand[c] >> 32, lo = cand[c] & 0xffffffffll;
  int32_t vid[4];
  if (!ee) {
    vid[0] = int32_t(hi);
    for (int j = 0; j < 3; ++j) vid[1 + j] = tris[3 * lo + j];
  } else {
    vid[0] = edges[2 * hi];
    vid[1] = edges[2 * hi + 1];
    vid[2] = edges[2 * lo];
    vid[3] = edges[2 * lo + 1];
  }
  double y[12];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) y[3 * a + i] = x[3 * int64_t(vid[a]) + i];
  const double d2 = ee ? ee_d2(y) : pt_d2(y);
  keep[c] = d2 < dhat2 ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_compact(int64_t nc, const int64_t* __restrict__ cand,
                                                 const int64_t* __restrict__ keep, const int64_t* __restrict__ pos,
                                                 int64_t* __restrict__ out) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc || !keep[c]) return;
  out[pos[c]] = cand[c];
}

// device buffers from the ms_device allocator, released on scope exit
struct Pool {
  const ms_device* dev;
  std::vector<void*> ptrs;
  explicit Pool(const ms_device* d) : dev(d) {}
  template <typename T>
  T* get(size_t n) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (dev->alloc)
      p = dev->alloc(bytes, dev->user);
    else if (hipMalloc(&p, bytes) != hipSuccess)
      p = nullptr;
    if (p) ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  ~Pool() {
    for (void* p : ptrs) {
      if (dev->free)
        dev->free(p, dev->user);
      else
        (void)hipFree(p);
    }
  }
};

inline unsigned blocks(int64_t n) { return unsigned((n + 255) / 256); }

// The pairs of one kind (vertex-triangle or edge-edge), sorted keys out:
// those closer than d_hat at x, or (x2 given, narrow false) every candidate
// whose swept boxes from x to x2 share a cell.
ms_status find_pairs(Pool& pool, hipStream_t st, bool ee, int64_t np_a, const int32_t* prims_a, int ka,
                     int64_t np_b, const int32_t* prims_b, int kb, const double* x, const int32_t* tris,
                     const int32_t* edges, double dhat, double inv_cell, std::vector<int64_t>& result,
                     const double* x2 = nullptr, bool narrow = true) {
  result.clear();
  const int64_t nprim = np_a + np_b;
  if (np_a == 0 || (!ee && np_b == 0)) return MS_OK;
  int64_t* cnt = pool.get<int64_t>(nprim + 1);
  int64_t* off = pool.get<int64_t>(nprim + 1);
  if (!cnt || !off) return MS_E_NOMEM;
  const double r = 0.5 * dhat;
  auto sync_read = [&](const int64_t* d, int64_t* h) -> bool {
    return hipMemcpyAsync(h, d, sizeof(int64_t), hipMemcpyDeviceToHost, st) == hipSuccess &&
           hipStreamSynchronize(st) == hipSuccess;
  };
  auto exclusive_scan = [&](const int64_t* in, int64_t* out, int64_t n) -> ms_status {
    size_t tmp = 0;
    if (rocprim::exclusive_scan(nullptr, tmp, in, out, int64_t(0), size_t(n), rocprim::plus<int64_t>(), st) !=
        hipSuccess)
      return MS_E_DEVICE;
    void* t = pool.get<char>(tmp);
    if (!t) return MS_E_NOMEM;
    if (rocprim::exclusive_scan(t, tmp, in, out, int64_t(0), size_t(n), rocprim::plus<int64_t>(), st) != hipSuccess)
      return MS_E_DEVICE;
    return MS_OK;
  };
  // entries: a-primitives, then b-primitives (tagged)
  if (hipMemsetAsync(cnt, 0, (nprim + 1) * sizeof(int64_t), st) != hipSuccess) return MS_E_DEVICE;
  k_cells<<<blocks(np_a), 256, 0, st>>>(np_a, prims_a, ka, x, x2, r, inv_cell, 0, 0, cnt, nullptr, nullptr,
                                        nullptr);
  if (np_b)
    k_cells<<<blocks(np_b), 256, 0, st>>>(np_b, prims_b, kb, x, x2, r, inv_cell, kTri, 0, cnt + np_a, nullptr,
                                          nullptr, nullptr);
  ms_status s;
  if ((s = exclusive_scan(cnt, off, nprim + 1))) return s;
  int64_t ne = 0;
  if (!sync_read(off + nprim, &ne)) return MS_E_DEVICE;
  if (ne >= (int64_t(1) << 31)) return MS_E_ARG;
  int64_t* keys = pool.get<int64_t>(ne);
  int64_t* vals = pool.get<int64_t>(ne);
  int64_t* skeys = pool.get<int64_t>(ne);
  int64_t* svals = pool.get<int64_t>(ne);
  int64_t* cend = pool.get<int64_t>(ne);
  if (!keys || !vals || !skeys || !svals || !cend) return MS_E_NOMEM;
  k_cells<<<blocks(np_a), 256, 0, st>>>(np_a, prims_a, ka, x, x2, r, inv_cell, 0, 1, nullptr, off, keys, vals);
  if (np_b)
    k_cells<<<blocks(np_b), 256, 0, st>>>(np_b, prims_b, kb, x, x2, r, inv_cell, kTri, 1, nullptr, off + np_a,
                                          keys, vals);
  {
    size_t tmp = 0;
    if (rocprim::radix_sort_pairs(nullptr, tmp, keys, skeys, vals, svals, ne, 0, 64, st) != hipSuccess)
      return MS_E_DEVICE;
    void* t = pool.get<char>(tmp);
    if (!t) return MS_E_NOMEM;
    if (rocprim::radix_sort_pairs(t, tmp, keys, skeys, vals, svals, ne, 0, 64, st) != hipSuccess)
      return MS_E_DEVICE;
  }
  k_cell_end<<<blocks(ne), 256, 0, st>>>(ne, skeys, cend);
  int64_t* ccnt = pool.get<int64_t>(ne + 1);
  int64_t* coff = pool.get<int64_t>(ne + 1);
  if (!ccnt || !coff) return MS_E_NOMEM;
  if (hipMemsetAsync(ccnt, 0, (ne + 1) * sizeof(int64_t), st) != hipSuccess) return MS_E_DEVICE;
  k_candidates<<<blocks(ne), 256, 0, st>>>(ne, skeys, svals, cend, ee ? 1 : 0, tris, edges, 0, ccnt, nullptr,
                                           nullptr);
  if ((s = exclusive_scan(ccnt, coff, ne + 1))) return s;
  int64_t nc = 0;
  if (!sync_read(coff + ne, &nc)) return MS_E_DEVICE;
  if (nc >= (int64_t(1) << 31)) return MS_E_ARG;
  if (nc == 0) return MS_OK;
  int64_t* cand = pool.get<int64_t>(nc);
  int64_t* scand = pool.get<int64_t>(nc);
  int64_t* ucand = pool.get<int64_t>(nc);
  int64_t* nu_d = pool.get<int64_t>(1);
  if (!cand || !scand || !ucand || !nu_d) return MS_E_NOMEM;
  k_candidates<<<blocks(ne), 256, 0, st>>>(ne, skeys, svals, cend, ee ? 1 : 0, tris, edges, 1, nullptr, coff,
                                           cand);
  {
    size_t tmp = 0;
    if (rocprim::radix_sort_keys(nullptr, tmp, cand, scand, nc, 0, 64, st) != hipSuccess)
      return MS_E_DEVICE;
    void* t = pool.get<char>(tmp);
    if (!t) return MS_E_NOMEM;
    if (rocprim::radix_sort_keys(t, tmp, cand, scand, nc, 0, 64, st) != hipSuccess) return MS_E_DEVICE;
  }
  {
    size_t tmp = 0;
    if (rocprim::unique(nullptr, tmp, scand, ucand, nu_d, size_t(nc), rocprim::equal_to<int64_t>(), st) != hipSuccess)
      return MS_E_DEVICE;
    void* t = pool.get<char>(tmp);
    if (!t) return MS_E_NOMEM;
    if (rocprim::unique(t, tmp, scand, ucand, nu_d, size_t(nc), rocprim::equal_to<int64_t>(), st) != hipSuccess)
      return MS_E_DEVICE;
  }
  int64_t nu = 0;
  if (!sync_read(nu_d, &nu)) return MS_E_DEVICE;
  if (nu == 0) return MS_OK;
  if (!narrow) {
    result.resize(nu);
    if (hipMemcpyAsync(result.data(), ucand, nu * sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return MS_E_DEVICE;
    return MS_OK;
  }
  int64_t* keep = pool.get<int64_t>(nu + 1);
  int64_t* pos = pool.get<int64_t>(nu + 1);
  int64_t* outd = pool.get<int64_t>(nu);
  if (!keep || !pos || !outd) return MS_E_NOMEM;
  if (hipMemsetAsync(keep, 0, (nu + 1) * sizeof(int64_t), st) != hipSuccess) return MS_E_DEVICE;
  k_narrow<<<blocks(nu), 256, 0, st>>>(nu, ucand, ee ? 1 : 0, x, tris, edges, dhat * dhat, keep);
  if ((s = exclusive_scan(keep, pos, nu + 1))) return s;
  int64_t nk = 0;
  if (!sync_read(pos + nu, &nk)) return MS_E_DEVICE;
  k_compact<<<blocks(nu), 256, 0, st>>>(nu, ucand, keep, pos, outd);
  result.resize(nk);
  if (nk > 0 && hipMemcpyAsync(result.data(), outd, nk * sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess)
    return MS_E_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return MS_E_DEVICE;
  return MS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Self-contact in the Newton step.  The constraint set at x comes from the
// grid broad phase above; the host turns its sorted pair keys into vertex
// quadruples and into gather lists (per vertex for the gradient, per Hessian
// slot for the curvature), so every sum runs in a fixed order.  Per pair:
//   E_p = h^2 kappa m(c) b(d),
//   grad E_p = h^2 kappa (m b'(d) grad d + m'(c) b(d) grad c),
//   H_p ~ h^2 kappa m b''(d) grad d grad d^T   (positive semi-definite),
// with m = 1 for point-triangle pairs.  The squared distance is a minimum of
// |p - closest point|^2 over the primitives' parameters; at its unique
// minimiser the gradient is the partial gradient there (Danskin's theorem):
// grad_a d^2 = 2 c_a r with r the difference of the closest points and c_a
// the signed barycentric weight of vertex a, hence grad_a d = c_a r / |r|.
// The curvature keeps only the barrier's second derivative along grad d (a
// Gauss-Newton form: the iterates change, the minimiser does not).
// ---------------------------------------------------------------------------
namespace {

// closest point of segment [a, b] to p: parameter t, r = p - closest, |r|^2
__device__ __forceinline__ double seg_closest(const double* p, const double* a, const double* b, double& t,
                                              double r[3]) {
  double ab[3], ap[3];
  sub3(b, a, ab);
  sub3(p, a, ap);
  t = fmin(fmax(dot3(ap, ab) / dot3(ab, ab), 0.0), 1.0);
  for (int i = 0; i < 3; ++i) r[i] = p[i] - (a[i] + t * ab[i]);
  return dot3(r, r);
}

// squared distance, r and the coefficients c_a of the four vertices (point,
// triangle vertices; or the two edges), with the same case split as pt_d2
// and ee_d2 (the first nearest segment wins ties)
__device__ double pair_geometry(bool ee, const double* y, double r[3], double cf[4]) {
  const double *p0 = y, *p1 = y + 3, *p2 = y + 6, *p3 = y + 9;
  if (!ee) {
    double e0[3], e1[3], w[3], n[3];
    sub3(p2, p1, e0);
    sub3(p3, p1, e1);
    sub3(p0, p1, w);
    cross3(e0, e1, n);
    const double d00 = dot3(e0, e0), d01 = dot3(e0, e1), d11 = dot3(e1, e1);
    const double d20 = dot3(w, e0), d21 = dot3(w, e1);
    const double den = d00 * d11 - d01 * d01;
    const double v = (d11 * d20 - d01 * d21) / den;
    const double u = (d00 * d21 - d01 * d20) / den;
    if (v >= 0.0 && u >= 0.0 && u + v <= 1.0) {
      const double h = dot3(w, n), nn = dot3(n, n);
      for (int i = 0; i < 3; ++i) r[i] = (h / nn) * n[i];
      cf[0] = 1.0;
      cf[1] = -(1.0 - u - v);
      cf[2] = -v;
      cf[3] = -u;
      return h * h / nn;
    }
    const double* sa[3] = {p1, p2, p1};
    const double* sb[3] = {p2, p3, p3};
    const int ia[3] = {1, 2, 1}, ib[3] = {2, 3, 3};
    double best = INFINITY;
    for (int k = 0; k < 3; ++k) {
      double t, rk[3];
      const double d2 = seg_closest(p0, sa[k], sb[k], t, rk);
      if (d2 < best) {
        best = d2;
        for (int i = 0; i < 3; ++i) r[i] = rk[i];
        cf[0] = 1.0;
        cf[1] = cf[2] = cf[3] = 0.0;
        cf[ia[k]] = -(1.0 - t);
        cf[ib[k]] = -t;
      }
    }
    return best;
  }
  double u[3], v[3], w[3];
  sub3(p1, p0, u);
  sub3(p3, p2, v);
  sub3(p0, p2, w);
  const double uu = dot3(u, u), uv = dot3(u, v), vv = dot3(v, v), uw = dot3(u, w), vw = dot3(v, w);
  const double den = uu * vv - uv * uv;
  if (den > 1e-12 * uu * vv) {
    const double sp = (uv * vw - vv * uw) / den;
    const double tq = (uu * vw - uv * uw) / den;
    if (sp >= 0.0 && sp <= 1.0 && tq >= 0.0 && tq <= 1.0) {
      double n[3];
      cross3(u, v, n);
      const double h = dot3(w, n), nn = dot3(n, n);
      for (int i = 0; i < 3; ++i) r[i] = (h / nn) * n[i];
      cf[0] = 1.0 - sp;
      cf[1] = sp;
      cf[2] = -(1.0 - tq);
      cf[3] = -tq;
      return h * h / nn;
    }
  }
  // endpoint against the other segment: a0, a1 against [b0, b1], then b0, b1 against [a0, a1]
  const double* pt[4] = {p0, p1, p2, p3};
  double best = INFINITY;
  for (int k = 0; k < 4; ++k) {
    const double* sa = k < 2 ? p2 : p0;
    const double* sb = k < 2 ? p3 : p1;
    double t, rk[3];
    const double d2 = seg_closest(pt[k], sa, sb, t, rk);
    if (d2 < best) {
      best = d2;
      for (int i = 0; i < 3; ++i) r[i] = rk[i];
      cf[0] = cf[1] = cf[2] = cf[3] = 0.0;
      cf[k] = 1.0;
      const int s0 = k < 2 ? 2 : 0;
      cf[s0] = -(1.0 - t);
      cf[s0 + 1] = -t;
    }
  }
  return best;
}

// mollifier of nearly parallel edges: m(c), m'(c) with c = |u x v|^2 and
// eps_x = 1e-3 |A1 - A0|^2 |B1 - B0|^2 at rest
__device__ __forceinline__ void mollifier(const double* y, const double* rest4, double& m, double& dm,
                                          double gc[12]) {
  double u[3], v[3], uv[3], ua[3], ub[3];
  sub3(y + 3, y, u);
  sub3(y + 9, y + 6, v);
  cross3(u, v, uv);
  const double c = dot3(uv, uv);
  double ru[3], rv[3];
  sub3(rest4 + 3, rest4, ru);
  sub3(rest4 + 9, rest4 + 6, rv);
  const double eps = 1e-3 * dot3(ru, ru) * dot3(rv, rv);
  if (c < eps) {
    const double q = c / eps;
    m = (2.0 - q) * q;
    dm = (2.0 - 2.0 * q) / eps;
  } else {
    m = 1.0;
    dm = 0.0;
  }
  cross3(v, uv, ua);  // grad_u c = 2 v x (u x v)
  cross3(uv, u, ub);  // grad_v c = 2 (u x v) x u
  for (int i = 0; i < 3; ++i) {
    gc[i] = -2.0 * ua[i];
    gc[3 + i] = 2.0 * ua[i];
    gc[6 + i] = -2.0 * ub[i];
    gc[9 + i] = 2.0 * ub[i];
  }
}

__device__ __forceinline__ void load_quad(const int32_t* __restrict__ quad, int64_t p, const double* __restrict__ x,
                                          const double* __restrict__ d, double alpha, double y[12], bool& ee) {
  ee = quad[5 * p] == 1;
  for (int a = 0; a < 4; ++a) {
    const int64_t v = quad[5 * p + 1 + a];
    for (int i = 0; i < 3; ++i) y[3 * a + i] = x[3 * v + i] + (d ? alpha * d[3 * v + i] : 0.0);
  }
}

// energy of one pair at positions y (kappa h^2 m b(d); 0 beyond d_hat)
__device__ double pair_energy(bool ee, const double* y, const double* rest4, double dhat, double kh2) {
  double r[3], cf[4];
  const double d2 = pair_geometry(ee, y, r, cf);
  if (!(d2 < dhat * dhat)) return 0.0;
  double b, b1, b2;
  barrier_terms(sqrt(d2), dhat, b, b1, b2);
  double m = 1.0;
  if (ee) {
    double dm, gc[12];
    mollifier(y, rest4, m, dm, gc);
  }
  return kh2 * m * b;
}

__device__ __forceinline__ void load_rest4(const int32_t* __restrict__ quad, int64_t p,
                                           const double* __restrict__ rest, double r4[12]) {
  for (int a = 0; a < 4; ++a) {
    const int64_t v = quad[5 * p + 1 + a];
    for (int i = 0; i < 3; ++i) r4[3 * a + i] = rest[3 * v + i];
  }
}

// per pair: [0] energy, [1..12] gradient, [13] Gauss-Newton weight,
// [14..17] coefficients c_a, [18..20] unit normal r / |r|
constexpr int kPd = 24;
__global__ void __launch_bounds__(256) k_sc_terms(int64_t np, const int32_t* __restrict__ quad,
                                                  const double* __restrict__ x, const double* __restrict__ rest,
                                                  double dhat, double kh2, double* __restrict__ pd) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= np) return;
  double y[12], r4[12];
  bool ee;
  load_quad(quad, p, x, nullptr, 0.0, y, ee);
  load_rest4(quad, p, rest, r4);
  double r[3], cf[4];
  const double d2 = pair_geometry(ee, y, r, cf);
  double* o = pd + kPd * p;
  for (int k = 0; k < kPd; ++k) o[k] = 0.0;
  if (!(d2 < dhat * dhat) || !(d2 > 0.0)) {
    if (!(d2 > 0.0)) o[0] = INFINITY;
    return;
  }
  const double dist = sqrt(d2);
  double b, b1, b2;
  barrier_terms(dist, dhat, b, b1, b2);
  double m = 1.0, dm = 0.0, gc[12];
  for (int k = 0; k < 12; ++k) gc[k] = 0.0;
  if (ee) mollifier(y, r4, m, dm, gc);
  const double rn = sqrt(dot3(r, r));
  double nh[3];
  for (int i = 0; i < 3; ++i) nh[i] = r[i] / rn;
  o[0] = kh2 * m * b;
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) o[1 + 3 * a + i] = kh2 * (m * b1 * cf[a] * nh[i] + dm * b * gc[3 * a + i]);
  o[13] = kh2 * m * b2;
  for (int a = 0; a < 4; ++a) o[14 + a] = cf[a];
  for (int i = 0; i < 3; ++i) o[18 + i] = nh[i];
}

// energies of the listed pairs at y = x + alpha d (mode 0: out [2p] = E(y));
// mode 1: out [2p] = E(y) - E(x), out [2p + 1] = |E(y)| + |E(x)|
__global__ void __launch_bounds__(256) k_sc_energy(int64_t np, const int32_t* __restrict__ quad,
                                                   const double* __restrict__ x, const double* __restrict__ d,
                                                   double alpha, const double* __restrict__ rest, double dhat,
                                                   double kh2, int mode, double* __restrict__ out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= np) return;
  double y[12], r4[12];
  bool ee;
  load_rest4(quad, p, rest, r4);
  load_quad(quad, p, x, d, alpha, y, ee);
  const double ey = pair_energy(ee, y, r4, dhat, kh2);
  if (mode == 0) {
    out[2 * p] = ey;
    out[2 * p + 1] = fabs(ey);
    return;
  }
  load_quad(quad, p, x, nullptr, 0.0, y, ee);
  const double ex = pair_energy(ee, y, r4, dhat, kh2);
  out[2 * p] = ey - ex;
  out[2 * p + 1] = fabs(ey) + fabs(ex);
}

// g_v += sum of the pair gradients of v's entries, in list order.  list:
// ng vertex ids, ng + 1 offsets, entries (pair, local vertex)
__global__ void __launch_bounds__(256) k_sc_grad(int64_t ng, const int32_t* __restrict__ list,
                                                 const double* __restrict__ pd, double* __restrict__ g) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= ng) return;
  const int64_t v = list[k];
  const int32_t* off = list + ng;
  const int32_t* ent = list + 2 * ng + 1;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = off[k]; e < off[k + 1]; ++e) {
    const double* o = pd + kPd * int64_t(ent[2 * e]) + 1 + 3 * ent[2 * e + 1];
    for (int i = 0; i < 3; ++i) acc[i] += o[i];
  }
  for (int i = 0; i < 3; ++i) g[3 * v + i] += acc[i];
}

// Hessian slot += sum over its entries (pair, a, b) of w c_a c_b n n^T.  list:
// nh slots, nh + 1 offsets, entries (pair, a, b)
template <typename VT>
__global__ void __launch_bounds__(256) k_sc_hess(int64_t nh, const int32_t* __restrict__ list,
                                                 const double* __restrict__ pd, int S, VT* __restrict__ vals) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nh) return;
  const int64_t slot = list[k];
  const int32_t* off = list + nh;
  const int32_t* ent = list + 2 * nh + 1;
  double acc[9];
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  for (int e = off[k]; e < off[k + 1]; ++e) {
    const double* o = pd + kPd * int64_t(ent[3 * e]);
    const double f = o[13] * o[14 + ent[3 * e + 1]] * o[14 + ent[3 * e + 2]];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) acc[3 * i + j] += f * o[18 + i] * o[18 + j];
  }
  VT* out = vals + vbase(slot, S);
  for (int q = 0; q < 9; ++q) out[S * q] = VT(double(out[S * q]) + acc[q]);
}

// additive CCD of each listed pair along x + t d, t in [0, 1] (as k_accd)
__global__ void __launch_bounds__(256) k_sc_accd(int64_t np, const int32_t* __restrict__ quad,
                                                 const double* __restrict__ x, const double* __restrict__ dd,
                                                 double s, int max_iter, double* __restrict__ toi) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= np) return;
  double y[12], p[12];
  bool ee;
  load_quad(quad, q, x, nullptr, 0.0, y, ee);
  load_quad(quad, q, dd, nullptr, 0.0, p, ee);
  const bool pt = !ee;
  double mean[3];
  for (int i = 0; i < 3; ++i) mean[i] = (p[i] + p[3 + i] + p[6 + i] + p[9 + i]) / 4.0;
  double nrm[4];
  for (int a = 0; a < 4; ++a) {
    for (int i = 0; i < 3; ++i) p[3 * a + i] -= mean[i];
    nrm[a] = sqrt(dot3(p + 3 * a, p + 3 * a));
  }
  const double lp = pt ? nrm[0] + fmax(fmax(nrm[1], nrm[2]), nrm[3]) : fmax(nrm[0], nrm[1]) + fmax(nrm[2], nrm[3]);
  toi[q] = 1.0;
  if (lp == 0.0) return;
  double dist = sqrt(pt ? pt_d2(y) : ee_d2(y));
  const double gap = s * dist;
  double t = 0.0, tl = (1.0 - s) * dist / lp;
  for (int it = 0; it < max_iter; ++it) {
    for (int k = 0; k < 12; ++k) y[k] += tl * p[k];
    dist = sqrt(pt ? pt_d2(y) : ee_d2(y));
    if (t > 0.0 && dist < gap) {
      toi[q] = t;
      return;
    }
    t += tl;
    if (t > 1.0) return;
    tl = 0.9 * dist / lp;
  }
  toi[q] = t;  // iteration cap: the time reached (still conservative)
}

__global__ void k_sc_axpy(int64_t len, const double* __restrict__ x, const double* __restrict__ d, double alpha,
                          double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < len) y[i] = x[i] + alpha * d[i];
}

// per block: max |d| over the components of the listed vertices
__global__ void __launch_bounds__(256) k_sc_maxd(int64_t nv, const int32_t* __restrict__ verts,
                                                 const double* __restrict__ d, double* __restrict__ part) {
  __shared__ double sh[256];
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double m = 0.0;
  if (k < nv) {
    const int64_t v = verts[k];
    m = fmax(fmax(fabs(d[3 * v]), fabs(d[3 * v + 1])), fabs(d[3 * v + 2]));
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// growable device buffer of the context
template <class T>
ms_status reserve(ms_ctx* c, T** p, int64_t* cap, int64_t need) {
  if (need <= *cap && *p) return MS_OK;
  const int64_t n = std::max<int64_t>(need, std::max<int64_t>(2 * *cap, 256));
  ms_status s = alloc_n(c, p, size_t(n));
  if (s) return s;
  *cap = n;
  return MS_OK;
}

// the constraint set (pt, ee keys) at device positions x, or with x2 the CCD
// candidates of the motion x -> x2
ms_status pairs_at(ms_ctx* c, const double* x, const double* x2, double cell, std::vector<int64_t>& pt,
                   std::vector<int64_t>& ee) {
  SelfContact& S = c->sc;
  Pool pool(&c->dev);
  const double dh = x2 ? 0.0 : S.dhat;
  const bool narrow = x2 == nullptr;
  ms_status s = find_pairs(pool, c->stream, false, int64_t(S.h_verts.size()), S.d_verts, 1,
                           int64_t(S.h_tris.size() / 3), S.d_tris, 3, x, S.d_tris, S.d_edges, dh, 1.0 / cell, pt, x2,
                           narrow);
  if (!s)
    s = find_pairs(pool, c->stream, true, int64_t(S.h_edges.size() / 2), S.d_edges, 2, 0, nullptr, 0, x, S.d_tris,
                   S.d_edges, dh, 1.0 / cell, ee, x2, narrow);
  (void)hipStreamSynchronize(c->stream);  // nothing in flight when the pool is released
  if (s == MS_E_NOMEM) return fail(c, s, "self-contact broad phase: out of device memory");
  if (s == MS_E_ARG) return fail(c, s, "self-contact broad phase: too many grid cells");
  if (s) return fail(c, s, "self-contact broad phase failed");
  return MS_OK;
}

// vertex quadruples [kind, v0..v3] of sorted keys (point-triangle first)
void quads_of(const SelfContact& S, const std::vector<int64_t>& pt, const std::vector<int64_t>& ee,
              std::vector<int32_t>& q) {
  q.clear();
  q.reserve(5 * (pt.size() + ee.size()));
  for (int64_t k : pt) {
    const int64_t v = k >> 32, t = k & 0xffffffffll;
    q.insert(q.end(), {0, int32_t(v), S.h_tris[3 * t], S.h_tris[3 * t + 1], S.h_tris[3 * t + 2]});
  }
  for (int64_t k : ee) {
    const int64_t i = k >> 32, j = k & 0xffffffffll;
    q.insert(q.end(), {1, S.h_edges[2 * i], S.h_edges[2 * i + 1], S.h_edges[2 * j], S.h_edges[2 * j + 1]});
  }
}

// sorted union of two ascending key lists
std::vector<int64_t> key_union(const std::vector<int64_t>& a, const std::vector<int64_t>& b) {
  std::vector<int64_t> u;
  u.reserve(a.size() + b.size());
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(u));
  return u;
}

ms_status upload_quads(ms_ctx* c, const std::vector<int32_t>& q) {
  SelfContact& S = c->sc;
  const int64_t np = int64_t(q.size() / 5);
  ms_status s;
  if ((s = reserve(c, &S.d_aux, &S.cap_aux, 5 * np + 5))) return s;
  if ((s = reserve(c, &S.d_aux_out, &S.cap_aux_out, 2 * np + 2))) return s;
  if (np) MS_HIP(hipMemcpyAsync(S.d_aux, q.data(), q.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  return MS_OK;
}

// the listed pairs' energy sums (mode 0: at x + alpha d; 1: difference to x)
ms_status pair_sums(ms_ctx* c, const std::vector<int32_t>& q, const double* x, const double* d, double alpha,
                    double h2, int mode, double* sum, double* mag) {
  SelfContact& S = c->sc;
  const int64_t np = int64_t(q.size() / 5);
  *sum = *mag = 0.0;
  if (np == 0) return MS_OK;
  ms_status s = upload_quads(c, q);
  if (s) return s;
  k_sc_energy<<<blocks(np), 256, 0, c->stream>>>(np, S.d_aux, x, d, alpha, c->d_rest, S.dhat, h2 * S.kappa, mode,
                                                  S.d_aux_out);
  std::vector<double> out(2 * np);
  MS_HIP(hipMemcpyAsync(out.data(), S.d_aux_out, 2 * np * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if ((s = sync(c))) return s;
  for (int64_t p = 0; p < np; ++p) {  // fixed order
    *sum += out[2 * p];
    *mag += out[2 * p + 1];
  }
  return MS_OK;
}

}  // namespace

ms_status sc_setup(ms_ctx* c) {
  SelfContact& S = c->sc;
  const int64_t T = c->T;
  // surface: the tet faces that belong to one tet only
  std::vector<std::array<int32_t, 3>> faces;
  faces.reserve(4 * T);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t* v = &c->h_tets[4 * t];
    const int32_t f[4][3] = {{v[1], v[2], v[3]}, {v[0], v[2], v[3]}, {v[0], v[1], v[3]}, {v[0], v[1], v[2]}};
    for (auto& g : f) {
      std::array<int32_t, 3> a = {g[0], g[1], g[2]};
      std::sort(a.begin(), a.end());
      faces.push_back(a);
    }
  }
  std::sort(faces.begin(), faces.end());
  S.h_tris.clear();
  for (size_t i = 0; i < faces.size();) {
    size_t j = i + 1;
    while (j < faces.size() && faces[j] == faces[i]) ++j;
    if (j - i == 1) S.h_tris.insert(S.h_tris.end(), faces[i].begin(), faces[i].end());
    i = j;
  }
  std::vector<std::array<int32_t, 2>> edges;
  for (size_t f = 0; f < S.h_tris.size() / 3; ++f) {
    const int32_t* t = &S.h_tris[3 * f];
    edges.push_back({t[0], t[1]});
    edges.push_back({t[1], t[2]});
    edges.push_back({t[0], t[2]});
  }
  std::sort(edges.begin(), edges.end());
  edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
  S.h_edges.clear();
  for (auto& e : edges) S.h_edges.insert(S.h_edges.end(), e.begin(), e.end());
  S.h_verts.assign(S.h_tris.begin(), S.h_tris.end());
  std::sort(S.h_verts.begin(), S.h_verts.end());
  S.h_verts.erase(std::unique(S.h_verts.begin(), S.h_verts.end()), S.h_verts.end());
  // grid cell: the largest primitive extent at rest plus d_hat
  double ext = 0.0;
  for (size_t f = 0; f < S.h_tris.size() / 3; ++f)
    for (int i = 0; i < 3; ++i) {
      double lo = INFINITY, hi = -INFINITY;
      for (int a = 0; a < 3; ++a) {
        const double v = c->h_rest[3 * int64_t(S.h_tris[3 * f + a]) + i];
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
      ext = std::max(ext, hi - lo);
    }
  S.cell = ext + S.dhat;
  ms_status s;
  if ((s = upload(c, &S.d_tris, S.h_tris.data(), S.h_tris.size()))) return s;
  if ((s = upload(c, &S.d_edges, S.h_edges.data(), S.h_edges.size()))) return s;
  if ((s = upload(c, &S.d_verts, S.h_verts.data(), S.h_verts.size()))) return s;
  if ((s = alloc_n(c, &S.d_y, 3 * c->n))) return s;
  return build_pattern(c);  // with the contact slots of the surface rows
}

ms_status sc_assemble(ms_ctx* c, const double* x, double h2, int prec) {
  SelfContact& S = c->sc;
  const Pattern& P = c->pat;
  std::vector<int64_t> kpt, kee;
  ms_status s = pairs_at(c, x, nullptr, S.cell, kpt, kee);
  if (s) return s;
  std::vector<int32_t> q;
  quads_of(S, kpt, kee, q);
  const int64_t np = int64_t(q.size() / 5);
  // contact slots: every row's couplings outside its mesh neighbourhood
  // take its reserved slots in order of first appearance
  for (int32_t v : S.h_verts)
    for (int k = 0; k < S.spare; ++k) S.h_col[P.h_slice_base[v / P.S] + int64_t(S.h_spare0[v] + k) * P.S + v % P.S] = -1;
  std::vector<int32_t> used(c->n, 0);
  auto slot_of = [&](int32_t row, int32_t col, int64_t* slot) -> bool {
    const int32_t* b = &P.h_col[P.h_row_ptr[row]];
    const int32_t* e = &P.h_col[P.h_row_ptr[row + 1]];
    const int32_t* it = std::lower_bound(b, e, col);
    const int64_t base = P.h_slice_base[row / P.S] + row % P.S;
    if (it != e && *it == col) {
      *slot = base + int64_t(it - b) * P.S;
      return true;
    }
    if (S.h_spare0[row] < 0) return false;
    for (int k = 0; k < used[row]; ++k) {
      const int64_t sl = base + int64_t(S.h_spare0[row] + k) * P.S;
      if (S.h_col[sl] == col) {
        *slot = sl;
        return true;
      }
    }
    if (used[row] >= S.spare) return false;
    const int64_t sl = base + int64_t(S.h_spare0[row] + used[row]++) * P.S;
    S.h_col[sl] = col;
    *slot = sl;
    return true;
  };
  std::vector<std::array<int32_t, 3>> gent;  // (vertex, pair, a)
  std::vector<std::array<int64_t, 4>> hent;  // (slot, pair, a, b)
  gent.reserve(4 * np);
  hent.reserve(16 * np);
  int64_t over = 0;  // couplings beyond the reserved slots
  for (int64_t p = 0; p < np; ++p)
    for (int a = 0; a < 4; ++a) {
      const int32_t va = q[5 * p + 1 + a];
      gent.push_back({va, int32_t(p), a});
      for (int b = 0; b < 4; ++b) {
        int64_t sl;
        if (!slot_of(va, q[5 * p + 1 + b], &sl)) {
          ++over;
          continue;
        }
        hent.push_back({sl, p, a, b});
      }
    }
  if (over) {
    int most = 0;  // the largest number of contact couplings of one row
    std::vector<std::vector<int32_t>> cols(c->n);
    for (int64_t p = 0; p < np; ++p)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const int32_t va = q[5 * p + 1 + a], vb = q[5 * p + 1 + b];
          const int32_t* lo = &P.h_col[P.h_row_ptr[va]];
          const int32_t* hi = &P.h_col[P.h_row_ptr[va + 1]];
          if (!std::binary_search(lo, hi, vb)) cols[va].push_back(vb);
        }
    for (auto& v : cols) {
      std::sort(v.begin(), v.end());
      most = std::max(most, int(std::unique(v.begin(), v.end()) - v.begin()));
    }
    return fail(c, MS_E_ARG, "a surface vertex couples to " + std::to_string(most) +
                                 " vertices outside its mesh neighbourhood; " + std::to_string(S.spare) +
                                 " contact slots are reserved (ms_set_self_contact)");
  }
  std::sort(gent.begin(), gent.end());
  std::sort(hent.begin(), hent.end());
  std::vector<int32_t> gl, hl;
  {
    std::vector<int32_t> vid, off{0}, ent;
    for (size_t k = 0; k < gent.size(); ++k) {
      if (k == 0 || gent[k][0] != gent[k - 1][0]) {
        if (k) off.push_back(int32_t(k));
        vid.push_back(gent[k][0]);
      }
      ent.push_back(gent[k][1]);
      ent.push_back(gent[k][2]);
    }
    if (!gent.empty()) off.push_back(int32_t(gent.size()));
    S.ng = int64_t(vid.size());
    gl = vid;
    gl.insert(gl.end(), off.begin(), off.end());
    gl.insert(gl.end(), ent.begin(), ent.end());
  }
  {
    std::vector<int32_t> sid, off{0}, ent;
    for (size_t k = 0; k < hent.size(); ++k) {
      if (k == 0 || hent[k][0] != hent[k - 1][0]) {
        if (k) off.push_back(int32_t(k));
        sid.push_back(int32_t(hent[k][0]));
      }
      ent.push_back(int32_t(hent[k][1]));
      ent.push_back(int32_t(hent[k][2]));
      ent.push_back(int32_t(hent[k][3]));
    }
    if (!hent.empty()) off.push_back(int32_t(hent.size()));
    S.nh = int64_t(sid.size());
    hl = sid;
    hl.insert(hl.end(), off.begin(), off.end());
    hl.insert(hl.end(), ent.begin(), ent.end());
  }
  S.np = np;
  if ((s = reserve(c, &S.d_quad, &S.cap_quad, int64_t(q.size()) + 5)) ||
      (s = reserve(c, &S.d_pdat, &S.cap_pdat, kPd * np + kPd)) ||
      (s = reserve(c, &S.d_glist, &S.cap_glist, int64_t(gl.size()) + 1)) ||
      (s = reserve(c, &S.d_hlist, &S.cap_hlist, int64_t(hl.size()) + 1)))
    return s;
  MS_HIP(hipMemcpyAsync(P.d_col, S.h_col.data(), S.h_col.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  if (np == 0) return sync(c);
  MS_HIP(hipMemcpyAsync(S.d_quad, q.data(), q.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  MS_HIP(hipMemcpyAsync(S.d_glist, gl.data(), gl.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  MS_HIP(hipMemcpyAsync(S.d_hlist, hl.data(), hl.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  k_sc_terms<<<blocks(np), 256, 0, c->stream>>>(np, S.d_quad, x, c->d_rest, S.dhat, h2 * S.kappa, S.d_pdat);
  k_sc_grad<<<blocks(S.ng), 256, 0, c->stream>>>(S.ng, S.d_glist, S.d_pdat, c->d_g);
  if (prec == MS_PREC_FP64)
    k_sc_hess<double><<<blocks(S.nh), 256, 0, c->stream>>>(S.nh, S.d_hlist, S.d_pdat, P.S, c->d_vals);
  else
    k_sc_hess<float><<<blocks(S.nh), 256, 0, c->stream>>>(S.nh, S.d_hlist, S.d_pdat, P.S, c->d_vals32);
  return sync(c);  // the host lists above are released on return
}

ms_status sc_energy(ms_ctx* c, const double* x, double h2, double* e) {
  std::vector<int64_t> kpt, kee;
  ms_status s = pairs_at(c, x, nullptr, c->sc.cell, kpt, kee);
  if (s) return s;
  std::vector<int32_t> q;
  quads_of(c->sc, kpt, kee, q);
  double mag;
  return pair_sums(c, q, x, nullptr, 0.0, h2, 0, e, &mag);
}

ms_status sc_energy_delta(ms_ctx* c, const double* x, const double* d, double alpha, double h2, double* dE,
                          double* err) {
  SelfContact& S = c->sc;
  k_sc_axpy<<<blocks(3 * c->n), 256, 0, c->stream>>>(3 * c->n, x, d, alpha, S.d_y);
  std::vector<int64_t> px, ex, py, ey;
  ms_status s = pairs_at(c, x, nullptr, S.cell, px, ex);
  if (!s) s = pairs_at(c, S.d_y, nullptr, S.cell, py, ey);
  if (s) return s;
  // every pair active at either end: its barrier vanishes where it is not
  std::vector<int32_t> q;
  quads_of(S, key_union(px, py), key_union(ex, ey), q);
  return pair_sums(c, q, x, d, alpha, h2, 1, dE, err);
}

ms_status sc_ccd(ms_ctx* c, const double* x, const double* d, double* t) {
  SelfContact& S = c->sc;
  *t = 1.0;
  const int64_t nv = int64_t(S.h_verts.size());
  if (nv == 0) return MS_OK;
  // grid cell: primitive extent + d_hat + the largest surface displacement
  const int64_t nb = (nv + 255) / 256;
  k_sc_maxd<<<unsigned(nb), 256, 0, c->stream>>>(nv, S.d_verts, d, c->d_part);
  std::vector<double> part(nb);
  MS_HIP(hipMemcpyAsync(part.data(), c->d_part, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  ms_status s = sync(c);
  if (s) return s;
  double dmax = 0.0;
  for (double v : part) dmax = std::max(dmax, v);
  if (!std::isfinite(dmax)) return fail(c, MS_E_NONFINITE, "non-finite search direction");
  if (dmax == 0.0) return MS_OK;
  k_sc_axpy<<<blocks(3 * c->n), 256, 0, c->stream>>>(3 * c->n, x, d, 1.0, S.d_y);
  std::vector<int64_t> kpt, kee;
  if ((s = pairs_at(c, x, S.d_y, S.cell + dmax, kpt, kee))) return s;
  std::vector<int32_t> q;
  quads_of(S, kpt, kee, q);
  const int64_t np = int64_t(q.size() / 5);
  if (np == 0) return MS_OK;
  if ((s = upload_quads(c, q))) return s;
  k_sc_accd<<<blocks(np), 256, 0, c->stream>>>(np, S.d_aux, x, d, 0.1, 100000, S.d_aux_out);
  std::vector<double> toi(np);
  MS_HIP(hipMemcpyAsync(toi.data(), S.d_aux_out, np * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if ((s = sync(c))) return s;
  for (double v : toi) *t = std::min(*t, v);
  return MS_OK;
}

}  // namespace ms

struct ms_pairs {
  std::vector<int64_t> pt, ee;
};

extern "C" ms_status ms_contact_pairs(const ms_device* dev, int64_t n_verts, const double* x, int64_t n_sverts,
                                      const int32_t* sverts, int64_t n_tris, const int32_t* tris, int64_t n_edges,
                                      const int32_t* edges, double dhat, double cell, ms_pairs** out) {
  if (!dev || !x || !out || n_verts < 1 || n_sverts < 0 || n_tris < 0 || n_edges < 0) return MS_E_ARG;
  if ((n_sverts && !sverts) || (n_tris && !tris) || (n_edges && !edges)) return MS_E_ARG;
  if (!(dhat > 0.0) || !std::isfinite(dhat) || !std::isfinite(cell)) return MS_E_ARG;
  if (n_verts >= (int64_t(1) << 31) || n_tris >= (int64_t(1) << 31) || n_edges >= (int64_t(1) << 31)) return MS_E_ARG;
  for (int64_t k = 0; k < 3 * n_verts; ++k)
    if (!std::isfinite(x[k])) return MS_E_NONFINITE;
  for (int64_t k = 0; k < n_sverts; ++k)
    if (sverts[k] < 0 || sverts[k] >= n_verts) return MS_E_ARG;
  for (int64_t k = 0; k < 3 * n_tris; ++k)
    if (tris[k] < 0 || tris[k] >= n_verts) return MS_E_ARG;
  for (int64_t k = 0; k < 2 * n_edges; ++k)
    if (edges[k] < 0 || edges[k] >= n_verts) return MS_E_ARG;
  // cell size: the largest primitive extent plus d_hat unless given
  double lo[3] = {x[0], x[1], x[2]}, hi[3] = {x[0], x[1], x[2]};
  for (int64_t v = 0; v < n_verts; ++v)
    for (int i = 0; i < 3; ++i) lo[i] = std::min(lo[i], x[3 * v + i]), hi[i] = std::max(hi[i], x[3 * v + i]);
  if (!(cell > 0.0)) {
    double ext = 0.0;
    auto grow = [&](const int32_t* vid, int k) {
      for (int i = 0; i < 3; ++i) {
        double a = x[3 * int64_t(vid[0]) + i], b = a;
        for (int j = 1; j < k; ++j) a = std::min(a, x[3 * int64_t(vid[j]) + i]), b = std::max(b, x[3 * int64_t(vid[j]) + i]);
        ext = std::max(ext, b - a);
      }
    };
    for (int64_t t = 0; t < n_tris; ++t) grow(tris + 3 * t, 3);
    for (int64_t e = 0; e < n_edges; ++e) grow(edges + 2 * e, 2);
    cell = ext + dhat;
  }
  double cells = 1.0;  // cells of the whole scene: bounds every primitive's count
  for (int i = 0; i < 3; ++i) {
    if (std::max(std::fabs(lo[i]), std::fabs(hi[i])) + dhat >= cell * double(ms::kCellBias - 2)) return MS_E_ARG;
    cells *= (hi[i] - lo[i] + dhat) / cell + 2.0;
  }
  if (cells >= double(int64_t(1) << 31)) return MS_E_ARG;
  if (hipSetDevice(dev->device) != hipSuccess) return MS_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(dev->hip_stream);
  ms::Pool pool(dev);
  double* xd = pool.get<double>(3 * n_verts);
  int32_t* sd = pool.get<int32_t>(n_sverts);
  int32_t* td = pool.get<int32_t>(3 * n_tris);
  int32_t* ed = pool.get<int32_t>(2 * n_edges);
  if (!xd || !sd || !td || !ed) return MS_E_NOMEM;
  if (hipMemcpyAsync(xd, x, 3 * n_verts * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      (n_sverts && hipMemcpyAsync(sd, sverts, n_sverts * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess) ||
      (n_tris && hipMemcpyAsync(td, tris, 3 * n_tris * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess) ||
      (n_edges && hipMemcpyAsync(ed, edges, 2 * n_edges * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess)) {
    (void)hipStreamSynchronize(st);  // nothing in flight when the pool is released
    return MS_E_DEVICE;
  }
  ms_pairs* res = new ms_pairs();
  const double inv_cell = 1.0 / cell;
  ms_status s = ms::find_pairs(pool, st, false, n_sverts, sd, 1, n_tris, td, 3, xd, td, ed, dhat, inv_cell, res->pt);
  if (!s) s = ms::find_pairs(pool, st, true, n_edges, ed, 2, 0, nullptr, 0, xd, td, ed, dhat, inv_cell, res->ee);
  (void)hipStreamSynchronize(st);
  if (s) {
    delete res;
    return s;
  }
  *out = res;
  return MS_OK;
}

extern "C" ms_status ms_pairs_get(const ms_pairs* p, int64_t* n_pt, int32_t* pt, int64_t* n_ee, int32_t* ee) {
  if (!p || !n_pt || !n_ee) return MS_E_ARG;
  *n_pt = int64_t(p->pt.size());
  *n_ee = int64_t(p->ee.size());
  if (pt)
    for (size_t k = 0; k < p->pt.size(); ++k) pt[2 * k] = int32_t(p->pt[k] >> 32), pt[2 * k + 1] = int32_t(p->pt[k] & 0xffffffff);
  if (ee)
    for (size_t k = 0; k < p->ee.size(); ++k) ee[2 * k] = int32_t(p->ee[k] >> 32), ee[2 * k + 1] = int32_t(p->ee[k] & 0xffffffff);
  return MS_OK;
}

extern "C" void ms_pairs_free(ms_pairs* p) { delete p; }

extern "C" ms_status ms_contact_toi(const ms_device* dev, int64_t n_pairs, const int32_t* kind, const double* x12,
                                    const double* p12, double s, double t_max, int32_t max_iter, double* toi,
                                    int32_t* hit) {
  if (!dev || n_pairs < 0 || (n_pairs > 0 && (!kind || !x12 || !p12 || !toi || !hit))) return MS_E_ARG;
  if (!(s > 0.0 && s < 1.0) || !(t_max > 0.0) || !std::isfinite(t_max) || max_iter < 1) return MS_E_ARG;
  if (n_pairs == 0) return MS_OK;
  if (n_pairs > (int64_t(1) << 31)) return MS_E_ARG;
  for (int64_t q = 0; q < n_pairs; ++q)
    if (kind[q] != 0 && kind[q] != 1) return MS_E_ARG;
  for (int64_t k = 0; k < 12 * n_pairs; ++k)
    if (!std::isfinite(x12[k]) || !std::isfinite(p12[k])) return MS_E_NONFINITE;
  if (hipSetDevice(dev->device) != hipSuccess) return MS_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(dev->hip_stream);
  void* bufs[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const size_t bytes[5] = {size_t(n_pairs) * sizeof(int32_t), 12 * size_t(n_pairs) * sizeof(double),
                           12 * size_t(n_pairs) * sizeof(double), size_t(n_pairs) * sizeof(double),
                           size_t(n_pairs) * sizeof(int32_t)};
  ms_status status = MS_OK;
  for (int b = 0; b < 5 && status == MS_OK; ++b) {
    if (dev->alloc)
      bufs[b] = dev->alloc(bytes[b], dev->user);
    else if (hipMalloc(&bufs[b], bytes[b]) != hipSuccess)
      bufs[b] = nullptr;
    if (!bufs[b]) status = MS_E_NOMEM;
  }
  if (status == MS_OK &&
      (hipMemcpyAsync(bufs[0], kind, bytes[0], hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(bufs[1], x12, bytes[1], hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(bufs[2], p12, bytes[2], hipMemcpyHostToDevice, st) != hipSuccess))
    status = MS_E_DEVICE;
  if (status == MS_OK) {
    const unsigned nb = unsigned((n_pairs + 255) / 256);
    ms::k_accd<<<nb, 256, 0, st>>>(n_pairs, static_cast<const int32_t*>(bufs[0]), static_cast<const double*>(bufs[1]),
                                   static_cast<const double*>(bufs[2]), s, t_max, int(max_iter),
                                   static_cast<double*>(bufs[3]), static_cast<int32_t*>(bufs[4]));
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(toi, bufs[3], bytes[3], hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(hit, bufs[4], bytes[4], hipMemcpyDeviceToHost, st) != hipSuccess)
      status = MS_E_DEVICE;
  }
  if (hipStreamSynchronize(st) != hipSuccess && status == MS_OK) status = MS_E_DEVICE;
  for (int b = 0; b < 5; ++b)
    if (bufs[b]) {
      if (dev->free)
        dev->free(bufs[b], dev->user);
      else
        (void)hipFree(bufs[b]);
    }
  return status;
}
