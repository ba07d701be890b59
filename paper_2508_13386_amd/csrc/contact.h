// Rigid half-space contact: the IPC log barrier of Sec. 3.1 on the signed
// distance of each vertex to the plane n . x = off.
#pragma once
#include <hip/hip_runtime.h>

#include "ms_internal.h"

namespace ms {

struct HalfSpace {
  double n[3];
  double off, dhat, kappa;
  int on;
};

// b(d) = -(d - dhat)^2 ln(d / dhat) for 0 < d < dhat, 0 beyond, +inf at or
// below zero; b1 = b', b2 = b''.
__device__ __forceinline__ void barrier_terms(double d, double dhat, double& b, double& b1, double& b2) {
  b = b1 = b2 = 0.0;
  if (d <= 0.0) {
    b = INFINITY;
    return;
  }
  if (d >= dhat) return;
  const double l = log(d / dhat), e = d - dhat;
  b = -e * e * l;
  b1 = -2.0 * e * l - e * e / d;
  b2 = -2.0 * l - 4.0 * e / d + (e * e) / (d * d);
}

inline HalfSpace hs_of(const ms_ctx* c) {
  HalfSpace h;
  for (int i = 0; i < 3; ++i) h.n[i] = c->hs_n[i];
  h.off = c->hs_off;
  h.dhat = c->hs_dhat;
  h.kappa = c->hs_kappa;
  h.on = c->has_hs ? 1 : 0;
  return h;
}

}  // namespace ms
