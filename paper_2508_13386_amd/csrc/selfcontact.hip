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
#include <cmath>
#include <vector>

#include <hipcub/hipcub.hpp>

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

// box of primitive q (k vertices), inflated by r, in cell coordinates
__device__ __forceinline__ void prim_cells(const double* __restrict__ x, const int32_t* __restrict__ vid, int k,
                                           double r, double inv_cell, int64_t lo[3], int64_t hi[3]) {
  for (int i = 0; i < 3; ++i) {
    double a = x[3 * int64_t(vid[0]) + i], b = a;
    for (int j = 1; j < k; ++j) {
      const double v = x[3 * int64_t(vid[j]) + i];
      a = fmin(a, v);
      b = fmax(b, v);
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
                                               const double* __restrict__ x, double r, double inv_cell,
                                               int64_t tag, int pass, int64_t* __restrict__ cnt,
                                               const int64_t* __restrict__ off, int64_t* __restrict__ keys,
                                               int64_t* __restrict__ vals) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= np) return;
  int64_t lo[3], hi[3];
  prim_cells(x, prims + int64_t(k) * q, k, r, inv_cell, lo, hi);
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

// The pairs of one kind (vertex-triangle or edge-edge), sorted keys out.
ms_status find_pairs(Pool& pool, hipStream_t st, bool ee, int64_t np_a, const int32_t* prims_a, int ka,
                     int64_t np_b, const int32_t* prims_b, int kb, const double* x, const int32_t* tris,
                     const int32_t* edges, double dhat, double inv_cell, std::vector<int64_t>& result) {
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
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, in, out, int(n), st) != hipSuccess) return MS_E_DEVICE;
    void* t = pool.get<char>(tmp);
    if (!t) return MS_E_NOMEM;
    if (hipcub::DeviceScan::ExclusiveSum(t, tmp, in, out, int(n), st) != hipSuccess) return MS_E_DEVICE;
    return MS_OK;
  };
  // entries: a-primitives, then b-primitives (tagged)
  if (hipMemsetAsync(cnt, 0, (nprim + 1) * sizeof(int64_t), st) != hipSuccess) return MS_E_DEVICE;
  k_cells<<<blocks(np_a), 256, 0, st>>>(np_a, prims_a, ka, x, r, inv_cell, 0, 0, cnt, nullptr, nullptr, nullptr);
  if (np_b)
    k_cells<<<blocks(np_b), 256, 0, st>>>(np_b, prims_b, kb, x, r, inv_cell, kTri, 0, cnt + np_a, nullptr, nullptr,
                                          nullptr);
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
  k_cells<<<blocks(np_a), 256, 0, st>>>(np_a, prims_a, ka, x, r, inv_cell, 0, 1, nullptr, off, keys, vals);
  if (np_b)
    k_cells<<<blocks(np_b), 256, 0, st>>>(np_b, prims_b, kb, x, r, inv_cell, kTri, 1, nullptr, off + np_a, keys,
                                          vals);
  {
    size_t tmp = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, keys, skeys, vals, svals, int(ne), 0, 64, st) != hipSuccess)
      return MS_E_DEVICE;
    void* t = pool.get<char>(tmp);
    if (!t) return MS_E_NOMEM;
    if (hipcub::DeviceRadixSort::SortPairs(t, tmp, keys, skeys, vals, svals, int(ne), 0, 64, st) != hipSuccess)
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
    if (hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, cand, scand, int(nc), 0, 64, st) != hipSuccess)
      return MS_E_DEVICE;
    void* t = pool.get<char>(tmp);
    if (!t) return MS_E_NOMEM;
    if (hipcub::DeviceRadixSort::SortKeys(t, tmp, cand, scand, int(nc), 0, 64, st) != hipSuccess) return MS_E_DEVICE;
  }
  {
    size_t tmp = 0;
    if (hipcub::DeviceSelect::Unique(nullptr, tmp, scand, ucand, nu_d, int(nc), st) != hipSuccess)
      return MS_E_DEVICE;
    void* t = pool.get<char>(tmp);
    if (!t) return MS_E_NOMEM;
    if (hipcub::DeviceSelect::Unique(t, tmp, scand, ucand, nu_d, int(nc), st) != hipSuccess) return MS_E_DEVICE;
  }
  int64_t nu = 0;
  if (!sync_read(nu_d, &nu)) return MS_E_DEVICE;
  if (nu == 0) return MS_OK;
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
