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
  // lagged friction (mu > 0): coefficient, smoothing length eps_v h and the
  // positions x^t at the start of the step (device)
  double mu, epsh;
  const double* xt;
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
  h.mu = c->has_hs ? c->hs_mu : 0.0;
  h.epsh = c->hs_epsv * c->step_h;
  h.xt = c->d_xt;
  return h;
}

// Lagged Coulomb friction of vertex v against the plane (the D term of the
// incremental potential, Sec. 3.1, in the IPC form):
//   D_v(y) = mu lambda_v f0(|u|),  u = P (y - x^t_v),  P = I - n n^T,
// with the normal force lambda_v = kappa |b'(d(x^t_v))| frozen at the start of
// the step and f0(s) = s for s >= eps_v h, else
// -s^3 / (3 (eps_v h)^2) + s^2 / (eps_v h) + eps_v h / 3.
// Returns mu lambda_v (0: no friction on this vertex) and u.
__device__ __forceinline__ double friction_setup(const HalfSpace& hs, int64_t v, const double y[3], double u[3]) {
  const double* xt = hs.xt + 3 * v;
  double b, b1, b2;
  barrier_terms(hs.n[0] * xt[0] + hs.n[1] * xt[1] + hs.n[2] * xt[2] - hs.off, hs.dhat, b, b1, b2);
  const double mulam = hs.mu * hs.kappa * fabs(b1);
  const double w[3] = {y[0] - xt[0], y[1] - xt[1], y[2] - xt[2]};
  const double wn = hs.n[0] * w[0] + hs.n[1] * w[1] + hs.n[2] * w[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) u[i] = w[i] - wn * hs.n[i];
  return mulam;
}

__device__ __forceinline__ double friction_f0(double s, double eh) {
  return s >= eh ? s : (-s * s * s / (3.0 * eh * eh) + s * s / eh + eh / 3.0);
}

// Energy, gradient and 3x3 Hessian of D_v at y (all zero without friction):
//   grad = mu lambda (f1/s) u,
//   Hess = mu lambda [(f1/s) P + (f0'' - f1/s) u u^T / s^2]   (PSD),
// with the rest limit (s -> 0) grad -> 0, Hess -> mu lambda (2/eh) P.
__device__ __forceinline__ double friction_terms(const HalfSpace& hs, int64_t v, const double y[3], double g[3],
                                                 double H[9]) {
  double u[3];
  const double mulam = friction_setup(hs, v, y, u);
  const double eh = hs.epsh;
  const double s = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double c1, c2;  // f1/s and (f0'' - f1/s)/s^2
  if (s >= eh) {
    c1 = 1.0 / s;
    c2 = -1.0 / (s * s * s);
  } else {
    c1 = -s / (eh * eh) + 2.0 / eh;
    c2 = s > 0.0 ? -1.0 / (eh * eh * s) : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) g[i] = mulam * c1 * u[i];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      H[3 * i + j] = mulam * (c1 * ((i == j ? 1.0 : 0.0) - hs.n[i] * hs.n[j]) + c2 * u[i] * u[j]);
  return mulam * friction_f0(s, eh);
}

// D_v(y) alone.
__device__ __forceinline__ double friction_energy(const HalfSpace& hs, int64_t v, const double y[3]) {
  double u[3];
  const double mulam = friction_setup(hs, v, y, u);
  if (mulam == 0.0) return 0.0;
  return mulam * friction_f0(sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]), hs.epsh);
}

}  // namespace ms
