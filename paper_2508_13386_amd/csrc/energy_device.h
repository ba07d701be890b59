// Per-item terms of the energy difference E(x + alpha d) - E(x) (see the
// kernel that sums them): one tet's elastic term and one vertex's inertia,
// gravity and barrier terms, each added into e[0..3] with their magnitudes
// in e[4].  Shared by the single-scene and the batched reductions so both
// evaluate the same arithmetic.
#pragma once
#include "contact.h"

namespace ms {

__device__ __forceinline__ void tet_energy_delta(int64_t i, const int32_t* __restrict__ tets,
                                               const double* __restrict__ Dminv, const double* __restrict__ vol,
                                               const double* __restrict__ mu_, const double* __restrict__ lam_,
                                               const double* __restrict__ x, const double* __restrict__ d,
                                               double alpha, double h2, double e[5]) {
  double F[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, D[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double b0[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) b0[j] = -(Dminv[9 * i + j] + Dminv[9 * i + 3 + j] + Dminv[9 * i + 6 + j]);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t v = tets[4 * i + a];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double y = x[3 * v + r], dy = alpha * d[3 * v + r];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double bj = a == 0 ? b0[j] : Dminv[9 * i + 3 * (a - 1) + j];
        F[r][j] += y * bj;
        D[r][j] += dy * bj;
      }
    }
  }
  double cF[3][3], cD[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int r1 = (r + 1) % 3, r2 = (r + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      cF[r][j] = F[r1][j1] * F[r2][j2] - F[r1][j2] * F[r2][j1];
      cD[r][j] = D[r1][j1] * D[r2][j2] - D[r1][j2] * D[r2][j1];
    }
  double FD = 0.0, DD = 0.0, cFD = 0.0, FcD = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      FD += F[r][j] * D[r][j];
      DD += D[r][j] * D[r][j];
      cFD += cF[r][j] * D[r][j];
      FcD += F[r][j] * cD[r][j];
    }
  const double J = F[0][0] * cF[0][0] + F[0][1] * cF[0][1] + F[0][2] * cF[0][2];
  const double detD = D[0][0] * cD[0][0] + D[0][1] * cD[0][1] + D[0][2] * cD[0][2];
  const double dIc = 2.0 * FD + DD;
  const double dJ = cFD + FcD + detD;
  const double mu = mu_[i], lam = lam_[i];
  e[1] = h2 * vol[i] * (0.5 * mu * dIc - mu * dJ + 0.5 * lam * dJ * (dJ + 2.0 * (J - 1.0)));
  e[4] = h2 * vol[i] * (0.5 * mu * (2.0 * fabs(FD) + DD) + mu * fabs(dJ) + 0.5 * lam * fabs(dJ) * (fabs(dJ) + 2.0 * fabs(J - 1.0)));
  }

__device__ __forceinline__ void vertex_energy_delta(int64_t i, const double* __restrict__ mass,
                                                  const double* __restrict__ x, const double* __restrict__ d,
                                                  double alpha, const double* __restrict__ xtilde, double h2,
                                                  double gx, double gy, double gz, HalfSpace hs, double e[5]) {
  const double m = mass[i];
  double dv[3], dot_xd = 0.0, dd = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    dv[r] = alpha * d[3 * i + r];
    dot_xd += dv[r] * (x[3 * i + r] - xtilde[3 * i + r]);
    dd += dv[r] * dv[r];
  }
  e[0] = m * (dot_xd + 0.5 * dd);
  e[2] = -h2 * m * (gx * dv[0] + gy * dv[1] + gz * dv[2]);
  e[4] += m * (fabs(dot_xd) + 0.5 * dd) + fabs(e[2]);
  if (hs.on && m > 0.0) {  // massless (isolated, padding) vertices carry no contact
    double b, b1, b2, bn, bn1, bn2;
    const double dist = hs.n[0] * x[3 * i] + hs.n[1] * x[3 * i + 1] + hs.n[2] * x[3 * i + 2] - hs.off;
    const double ddist = hs.n[0] * dv[0] + hs.n[1] * dv[1] + hs.n[2] * dv[2];
    barrier_terms(dist, hs.dhat, b, b1, b2);
    barrier_terms(dist + ddist, hs.dhat, bn, bn1, bn2);
    e[3] = h2 * hs.kappa * (bn - b);
    e[4] += h2 * hs.kappa * (fabs(bn) + fabs(b));
    if (hs.mu > 0.0) {  // lagged friction: D_v(x + alpha d) - D_v(x)
      const double y0[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
      const double y1[3] = {y0[0] + dv[0], y0[1] + dv[1], y0[2] + dv[2]};
      const double f0 = friction_energy(hs, i, y0), f1 = friction_energy(hs, i, y1);
      e[3] += h2 * (f1 - f0);
      e[4] += h2 * (fabs(f1) + fabs(f0));
    }
  }
  }

}  // namespace ms
