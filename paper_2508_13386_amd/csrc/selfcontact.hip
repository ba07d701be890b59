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
#include <cmath>

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

}  // namespace
}  // namespace ms

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
