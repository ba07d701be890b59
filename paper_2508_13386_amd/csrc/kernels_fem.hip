// Element and assembly kernels of the incremental potential (Eq. IP, Sec. 3.1)
// for implicit Euler: stable Neo-Hookean elasticity per tet, lumped inertia,
// gravity, IPC half-space log barrier.
//
//   k_element      one thread per tet: F = sum_a x_a beta_a^T, the energy
//                  gradient (FP64) and the 12x12 Hessian V beta^T Pi beta,
//                  where Pi is d2Psi/dF2 (9x9) with its negative eigenvalues
//                  clamped to zero, or replaced by their absolute values
//                  (cyclic Jacobi in registers); stores the
//                  10 upper 3x3 blocks per tet (FP64 or FP32)
//   k_gather_grad  one thread per vertex, sums its incident tets' gradient
//                  blocks in tet order and adds inertia, gravity, barrier
//   k_gather_hess  one thread per Hessian slot, sums its element blocks in
//                  tet order (no atomics), scales by h^2, adds mass and
//                  barrier curvature on diagonal slots
//   k_energy       E(x + alpha d) parts with a deterministic grid reduction
//   k_ccd          largest safe step toward the half-space
#include <cfloat>

#include "contact.h"
#include "energy_device.h"
#include "ms_internal.h"
#include "reduce.h"

namespace ms {

__device__ __forceinline__ double sgn_cyc(int a, int b) {  // eps_{a b k} for k = 3-a-b
  return ((b - a + 3) % 3 == 1) ? 1.0 : -1.0;
}

// Packed upper-triangular index of a symmetric 9x9 matrix.
__host__ __device__ constexpr int ut(int i, int j) {
  return i <= j ? (i * 9 - (i * (i - 1)) / 2 + (j - i)) : (j * 9 - (j * (j - 1)) / 2 + (i - j));
}

// Deformation-gradient Hessian of the stable Neo-Hookean density,
//   C = mu I + lam' vec(cof F) vec(cof F)^T + (lam'(J-1) - mu) d2J/dF2,
// with d2J/dF_ip dF_jq = eps_ijk eps_pqr F_kr; packed upper triangle.
__device__ __forceinline__ void snh_hessian(const double F[3][3], const double cof[3][3], double J, double mu,
                                            double lam, double a[45]) {
  const double s = lam * (J - 1.0) - mu;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int r = 3 * i + p, cidx = 3 * j + q;
          if (cidx < r) continue;
          double v = lam * cof[i][p] * cof[j][q];
          if (r == cidx) v += mu;
          if (i != j && p != q) v += s * sgn_cyc(i, j) * sgn_cyc(p, q) * F[3 - i - j][3 - p - q];
          a[ut(r, cidx)] = v;
        }
}

// Cyclic Jacobi eigen-decomposition of the packed symmetric 9x9 matrix a;
// on return the diagonal of a holds the eigenvalues and the columns of V
// the eigenvectors.
__device__ __forceinline__ void jacobi9(double a[45], double V[9][9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 9; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = 0.0, dg = 0.0;
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      dg += a[ut(p, p)] * a[ut(p, p)];
#pragma unroll
      for (int q = p + 1; q < 9; ++q) off += a[ut(p, q)] * a[ut(p, q)];
    }
    if (off <= 1e-32 * dg || off == 0.0) break;
#pragma unroll
    for (int p = 0; p < 9; ++p)
#pragma unroll
      for (int q = p + 1; q < 9; ++q) {
        const double apq = a[ut(p, q)];
        if (apq == 0.0) continue;
        const double theta = (a[ut(q, q)] - a[ut(p, p)]) / (2.0 * apq);
        double t;
        if (fabs(theta) > 1e100) {
          t = 0.5 / theta;
        } else {
          t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
          if (theta < 0.0) t = -t;
        }
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        a[ut(p, p)] -= t * apq;
        a[ut(q, q)] += t * apq;
        a[ut(p, q)] = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          if (k == p || k == q) continue;
          const double akp = a[ut(k, p)], akq = a[ut(k, q)];
          a[ut(k, p)] = cs * akp - sn * akq;
          a[ut(k, q)] = sn * akp + cs * akq;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = cs * vkp - sn * vkq;
          V[k][q] = sn * vkp + cs * vkq;
        }
      }
  }
}

template <bool HESS, typename HT>
__global__ void __launch_bounds__(64) k_element(int64_t T, const int32_t* __restrict__ tets,
                                                const double* __restrict__ Dminv, const double* __restrict__ vol,
                                                const double* __restrict__ mu_, const double* __restrict__ lam_,
                                                const double* __restrict__ x, double* __restrict__ ge,
                                                HT* __restrict__ He, int project,
                                                const int32_t* __restrict__ tscene,
                                                const uint8_t* __restrict__ sproj) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= T) return;
  int vi[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) vi[a] = tets[4 * t + a];
  double X[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) X[a][i] = x[3 * int64_t(vi[a]) + i];
  double beta[4][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    beta[1][j] = Dminv[9 * t + 0 + j];
    beta[2][j] = Dminv[9 * t + 3 + j];
    beta[3][j] = Dminv[9 * t + 6 + j];
    beta[0][j] = -(beta[1][j] + beta[2][j] + beta[3][j]);
  }
  const double V = vol[t], mu = mu_[t], lam = lam_[t];
  double F[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) s += X[a][i] * beta[a][j];
      F[i][j] = s;
    }
  // cofactor columns: cof[:,0] = f1 x f2, cof[:,1] = f2 x f0, cof[:,2] = f0 x f1
  double cof[3][3];
#pragma unroll
  for (int col = 0; col < 3; ++col) {
    const int c1 = (col + 1) % 3, c2 = (col + 2) % 3;
    cof[0][col] = F[1][c1] * F[2][c2] - F[2][c1] * F[1][c2];
    cof[1][col] = F[2][c1] * F[0][c2] - F[0][c1] * F[2][c2];
    cof[2][col] = F[0][c1] * F[1][c2] - F[1][c1] * F[0][c2];
  }
  const double J = F[0][0] * cof[0][0] + F[1][0] * cof[1][0] + F[2][0] * cof[2][0];
  const double s = lam * (J - 1.0) - mu;
  double P[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) P[i][j] = mu * F[i][j] + s * cof[i][j];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double g = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) g += P[i][j] * beta[a][j];
      ge[12 * t + 3 * a + i] = V * g;
    }
  if (!HESS) return;
  double A[45];
  snh_hessian(F, cof, J, mu, lam, A);
  // per-scene choice in a batch: scene of the tet, then that scene's flag
  if (tscene ? sproj[tscene[t]] != 0 : project != 0) {
    double Q[9][9];
    jacobi9(A, Q);
    double lp[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) lp[k] = project == 2 ? fabs(A[ut(k, k)]) : fmax(A[ut(k, k)], 0.0);
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
      for (int j = i; j < 9; ++j) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) v += Q[i][k] * lp[k] * Q[j][k];
        A[ut(i, j)] = v;
      }
  }
  // 10 stored blocks (a <= b): H[(a,i),(b,j)] = V sum_pq beta_a[p] C[(i,p),(j,q)] beta_b[q]
  HT* out = He + 90 * t;
  int pr = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            double w = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) w += A[ut(3 * i + p, 3 * j + q)] * beta[b][q];
            v += beta[a][p] * w;
          }
          out[9 * pr + 3 * i + j] = HT(V * v);
        }
      ++pr;
    }
}

__global__ void k_gather_grad(int64_t n, const int32_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt_code,
                              const double* __restrict__ ge, const double* __restrict__ mass,
                              const double* __restrict__ x, const double* __restrict__ xtilde, double h2, double gx,
                              double gy, double gz, HalfSpace hs, double* __restrict__ g) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const int k1 = vt_ptr[v + 1];
  for (int kb = vt_ptr[v]; kb < k1; kb += 8) {
    int code[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) code[u] = (kb + u < k1) ? vt_code[kb + u] : -1;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (code[u] < 0) continue;
      const double* p = ge + 12 * int64_t(code[u] >> 2) + 3 * (code[u] & 3);
      s0 += p[0];
      s1 += p[1];
      s2 += p[2];
    }
  }
  const double m = mass[v];
  const double x0 = x[3 * v], x1 = x[3 * v + 1], x2 = x[3 * v + 2];
  double r0 = m * (x0 - xtilde[3 * v]) + h2 * (s0 - m * gx);
  double r1 = m * (x1 - xtilde[3 * v + 1]) + h2 * (s1 - m * gy);
  double r2 = m * (x2 - xtilde[3 * v + 2]) + h2 * (s2 - m * gz);
  if (hs.on && m > 0.0) {  // massless (isolated, padding) vertices carry no contact
    double b, b1, b2;
    barrier_terms(hs.n[0] * x0 + hs.n[1] * x1 + hs.n[2] * x2 - hs.off, hs.dhat, b, b1, b2);
    const double f = h2 * hs.kappa * b1;
    r0 += f * hs.n[0];
    r1 += f * hs.n[1];
    r2 += f * hs.n[2];
    if (hs.mu > 0.0) {
      const double y[3] = {x0, x1, x2};
      double gf[3], Hf[9];
      friction_terms(hs, v, y, gf, Hf);
      r0 += h2 * gf[0];
      r1 += h2 * gf[1];
      r2 += h2 * gf[2];
    }
  }
  g[3 * v] = r0;
  g[3 * v + 1] = r1;
  g[3 * v + 2] = r2;
}

// grid: x = slice, y = group of 64/S block columns; lane = (column in group) * S + row
template <typename HT, typename VT>
__global__ void __launch_bounds__(64) k_gather_hess(int64_t n, int S, const int32_t* __restrict__ slice_base,
                                                    const int32_t* __restrict__ scol,
                                                    const int32_t* __restrict__ gptr,
                                                    const int32_t* __restrict__ gcode, const HT* __restrict__ He,
                                                    const double* __restrict__ mass, const double* __restrict__ x,
                                                    double h2, HalfSpace hs, VT* __restrict__ vals) {
  const int s = blockIdx.x, lane = threadIdx.x % S, k = blockIdx.y * (64 / S) + threadIdx.x / S;
  const int base = slice_base[s];
  const int width = (slice_base[s + 1] - base) / S;
  if (k >= width) return;
  const int64_t slot = int64_t(base) + int64_t(k) * S + lane;
  const int64_t row = int64_t(s) * S + lane;
  const int col = scol[slot];
  double acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = 0.0;
  if (col >= 0) {
    for (int e = gptr[slot]; e < gptr[slot + 1]; ++e) {
      const int code = gcode[e];
      const HT* blk = He + 9 * int64_t(code >> 1);
      if (code & 1) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) acc[3 * i + j] += double(blk[3 * j + i]);
      } else {
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[c] += double(blk[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] *= h2;
    if (col == row) {
      const double m = mass[row];
      acc[0] += m;
      acc[4] += m;
      acc[8] += m;
      if (hs.on && m > 0.0) {
        double b, b1, b2;
        barrier_terms(hs.n[0] * x[3 * row] + hs.n[1] * x[3 * row + 1] + hs.n[2] * x[3 * row + 2] - hs.off,
                      hs.dhat, b, b1, b2);
        const double f = h2 * hs.kappa * b2;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) acc[3 * i + j] += f * hs.n[i] * hs.n[j];
        if (hs.mu > 0.0) {
          const double y[3] = {x[3 * row], x[3 * row + 1], x[3 * row + 2]};
          double gf[3], Hf[9];
          friction_terms(hs, row, y, gf, Hf);
#pragma unroll
          for (int q = 0; q < 9; ++q) acc[q] += h2 * Hf[q];
        }
      }
    }
  }
  VT* out = vals + vbase(slot, S);
#pragma unroll
  for (int c = 0; c < 9; ++c) out[S * c] = VT(acc[c]);
}

// Energy parts at y = x + alpha d: {K, h^2 Psi, h^2 G, h^2 (B + D)} with D
// the lagged friction (zero unless mu > 0); threads cover
// max(T, n) indices, doing one tet and one vertex each.
__global__ void __launch_bounds__(256) k_energy(int64_t T, int64_t n, const int32_t* __restrict__ tets,
                                                const double* __restrict__ Dminv, const double* __restrict__ vol,
                                                const double* __restrict__ mu_, const double* __restrict__ lam_,
                                                const double* __restrict__ mass, const double* __restrict__ x,
                                                const double* __restrict__ d, double alpha,
                                                const double* __restrict__ xtilde, double h2, double gx, double gy,
                                                double gz, HalfSpace hs, double* __restrict__ part,
                                                unsigned* __restrict__ counter, double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double e[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < T) {
    double F[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double b0[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) b0[j] = -(Dminv[9 * i + j] + Dminv[9 * i + 3 + j] + Dminv[9 * i + 6 + j]);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t v = tets[4 * i + a];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double y = x[3 * v + r] + (d ? alpha * d[3 * v + r] : 0.0);
#pragma unroll
        for (int j = 0; j < 3; ++j) F[r][j] += y * (a == 0 ? b0[j] : Dminv[9 * i + 3 * (a - 1) + j]);
      }
    }
    const double J = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                     F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                     F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
    double Ic = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ic += F[r][j] * F[r][j];
    const double mu = mu_[i], lam = lam_[i];
    e[1] = h2 * vol[i] * (0.5 * mu * (Ic - 3.0) - mu * (J - 1.0) + 0.5 * lam * (J - 1.0) * (J - 1.0));
  }
  if (i < n) {
    const double m = mass[i];
    double y[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) y[r] = x[3 * i + r] + (d ? alpha * d[3 * i + r] : 0.0);
    const double d0 = y[0] - xtilde[3 * i], d1 = y[1] - xtilde[3 * i + 1], d2 = y[2] - xtilde[3 * i + 2];
    e[0] = 0.5 * m * (d0 * d0 + d1 * d1 + d2 * d2);
    e[2] = -h2 * m * (gx * y[0] + gy * y[1] + gz * y[2]);
    if (hs.on && m > 0.0) {
      double b, b1, b2;
      barrier_terms(hs.n[0] * y[0] + hs.n[1] * y[1] + hs.n[2] * y[2] - hs.off, hs.dhat, b, b1, b2);
      e[3] = h2 * hs.kappa * b;
      if (hs.mu > 0.0) e[3] += h2 * friction_energy(hs, i, y);
    }
  }
  if (grid_sum<4>(e, part, counter) && threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = e[k];
}

// E(x + alpha d) - E(x) by parts, written so that no large totals cancel:
//   inertia   sum_v m_v (alpha d_v.(x_v - x~_v) + alpha^2 |d_v|^2 / 2)
//   gravity   -h^2 alpha sum_v m_v g.d_v
//   elastic   per tet with delta = alpha grad(d) and F = grad(x):
//             dIc = 2 F:delta + |delta|^2,
//             dJ  = cof(F):delta + F:cof(delta) + det(delta)  (exact for 3x3),
//             dPsi = mu/2 dIc - mu dJ + lam/2 dJ (dJ + 2 (J - 1))
//   barrier   per vertex b(d') - b(d); lagged friction D_v(y') - D_v(y)
// out[4] = sum of the magnitudes of the terms above, the scale of the
// round-off in the total.  Threads cover max(T, n) indices, one tet and one vertex each.
__global__ void __launch_bounds__(256) k_energy_delta(int64_t T, int64_t n, const int32_t* __restrict__ tets,
                                                      const double* __restrict__ Dminv, const double* __restrict__ vol,
                                                      const double* __restrict__ mu_, const double* __restrict__ lam_,
                                                      const double* __restrict__ mass, const double* __restrict__ x,
                                                      const double* __restrict__ d, double alpha,
                                                      const double* __restrict__ xtilde, double h2, double gx,
                                                      double gy, double gz, HalfSpace hs, double* __restrict__ part,
                                                      unsigned* __restrict__ counter, double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double e[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < T) tet_energy_delta(i, tets, Dminv, vol, mu_, lam_, x, d, alpha, h2, e);
  if (i < n) vertex_energy_delta(i, mass, x, d, alpha, xtilde, h2, gx, gy, gz, hs, e);
  if (grid_sum<5>(e, part, counter) && threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) out[k] = e[k];
}

// Largest alpha in (0, 1] with every vertex kept at least (1 - safety) of its
// distance away from the plane: min over approaching vertices of
// safety * dist / (-n . d).
__global__ void __launch_bounds__(256) k_ccd(int64_t n, const double* __restrict__ x, const double* __restrict__ d,
                                             HalfSpace hs, double safety, double* __restrict__ part,
                                             unsigned* __restrict__ counter, double* __restrict__ out) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double a = 1.0;
  if (v < n) {
    const double dist = hs.n[0] * x[3 * v] + hs.n[1] * x[3 * v + 1] + hs.n[2] * x[3 * v + 2] - hs.off;
    const double app = -(hs.n[0] * d[3 * v] + hs.n[1] * d[3 * v + 1] + hs.n[2] * d[3 * v + 2]);
    if (app > 0.0) a = fmin(a, safety * dist / app);
  }
  // min-reduction through the sum machinery: reduce per block, then the
  // last block takes the minimum over partials
  __shared__ double sh[4];
  __shared__ int last;
  a = wave_min(a);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sh[0];
    for (int w = 1; w < int(blockDim.x >> 6); ++w) m = fmin(m, sh[w]);
    store_coherent(&part[blockIdx.x], m);
    __threadfence();
    last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) {
    double m = 1.0;
    for (unsigned b = 0; b < gridDim.x; ++b) m = fmin(m, load_coherent(&part[b]));
    out[0] = m;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_predict(int64_t n3, const double* __restrict__ x, const double* __restrict__ v, double h,
                          double* __restrict__ xt, double* __restrict__ xtilde) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  xt[i] = x[i];
  xtilde[i] = x[i] + h * v[i];
}

__global__ void k_apply_dbc(int64_t nd, const int32_t* __restrict__ idx, const double* __restrict__ tgt,
                            double* __restrict__ x) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nd) return;
  const int64_t v = idx[i];
  x[3 * v] = tgt[3 * i];
  x[3 * v + 1] = tgt[3 * i + 1];
  x[3 * v + 2] = tgt[3 * i + 2];
}

// d = x~ - x on free vertices, 0 on pinned ones.
__global__ void k_predictor_dir(int64_t n, const double* __restrict__ x, const double* __restrict__ xtilde,
                                const uint8_t* __restrict__ pinned, double* __restrict__ d) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const bool pin = pinned[v];
#pragma unroll
  for (int i = 0; i < 3; ++i) d[3 * v + i] = pin ? 0.0 : xtilde[3 * v + i] - x[3 * v + i];
}

__global__ void k_velocity(int64_t n3, const double* __restrict__ x, const double* __restrict__ xt, double inv_h,
                           double* __restrict__ v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  v[i] = (x[i] - xt[i]) * inv_h;
}

// BDF2 predictor: x^t kept, x~ = 4/3 x^t - 1/3 x^{t-1} + h (8 v^t - 2 v^{t-1}) / 9.
__global__ void k_predict_bdf2(int64_t n3, const double* __restrict__ x, const double* __restrict__ v,
                               const double* __restrict__ xprev, const double* __restrict__ vprev, double h,
                               double* __restrict__ xt, double* __restrict__ xtilde) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  xt[i] = x[i];
  xtilde[i] = (4.0 * x[i] - xprev[i]) / 3.0 + h * (8.0 * v[i] - 2.0 * vprev[i]) / 9.0;
}

// End of a step: v^{t+1} ((x - x^t)/h, or (3x - 4x^t + x^{t-1})/(2h) for
// BDF2) and the history shift x^{t-1} <- x^t, v^{t-1} <- v^t.
__global__ void k_velocity_hist(int64_t n3, const double* __restrict__ x, const double* __restrict__ xt,
                                double* __restrict__ xprev, double* __restrict__ v, double* __restrict__ vprev,
                                double inv_h, int bdf2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  const double vold = v[i], xp = xprev[i], xo = xt[i];
  // the implicit-Euler form is the one of k_velocity (same rounding as the
  // batched steps)
  v[i] = bdf2 ? (3.0 * x[i] - 4.0 * xo + xp) * (0.5 * inv_h) : (x[i] - xo) * inv_h;
  xprev[i] = xo;
  vprev[i] = vold;
}

static inline unsigned nblocks(int64_t n, int b) { return unsigned((n + b - 1) / b); }


void launch_predict(ms_ctx* c, double dt) {
  c->step_h = dt;  // the friction smoothing length eps_v h uses it
  k_predict<<<nblocks(3 * c->n, 256), 256, 0, c->stream>>>(3 * c->n, c->d_x, c->d_v, dt, c->d_xt, c->d_xtilde);
}
void launch_predict_bdf2(ms_ctx* c, double dt) {
  c->step_h = dt;
  k_predict_bdf2<<<nblocks(3 * c->n, 256), 256, 0, c->stream>>>(3 * c->n, c->d_x, c->d_v, c->d_xprev, c->d_vprev, dt,
                                                                c->d_xt, c->d_xtilde);
}
void launch_velocity_hist(ms_ctx* c, double dt, bool bdf2) {
  k_velocity_hist<<<nblocks(3 * c->n, 256), 256, 0, c->stream>>>(3 * c->n, c->d_x, c->d_xt, c->d_xprev, c->d_v,
                                                                 c->d_vprev, 1.0 / dt, bdf2 ? 1 : 0);
}
void launch_apply_dbc(ms_ctx* c, int64_t nd) {
  if (nd == 0) return;
  k_apply_dbc<<<nblocks(nd, 256), 256, 0, c->stream>>>(nd, c->d_dbc, c->d_dbc_tgt, c->d_x);
}
void launch_predictor_dir(ms_ctx* c) {
  k_predictor_dir<<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, c->d_x, c->d_xtilde, c->d_pinned, c->d_d);
}
void launch_velocity(ms_ctx* c, double inv_h) {
  k_velocity<<<nblocks(3 * c->n, 256), 256, 0, c->stream>>>(3 * c->n, c->d_x, c->d_xt, inv_h, c->d_v);
}
void launch_element(ms_ctx* c, const double* x, double /*h2*/, int prec, bool hess, bool proj,
                    const int32_t* tscene, const uint8_t* sproj) {
  const unsigned nb = nblocks(c->T, 64);
  const int project = proj ? (c->proj_mode == 1 ? 2 : 1) : 0;  // 2: absolute values
  if (!hess)
    k_element<false, double><<<nb, 64, 0, c->stream>>>(c->T, c->d_tets, c->d_Dminv, c->d_vol, c->d_mu, c->d_lam, x,
                                                      c->d_ge, c->d_He, project, tscene, sproj);
  else if (prec == MS_PREC_FP64)
    k_element<true, double><<<nb, 64, 0, c->stream>>>(c->T, c->d_tets, c->d_Dminv, c->d_vol, c->d_mu, c->d_lam, x,
                                                     c->d_ge, c->d_He, project, tscene, sproj);
  else
    k_element<true, float><<<nb, 64, 0, c->stream>>>(c->T, c->d_tets, c->d_Dminv, c->d_vol, c->d_mu, c->d_lam, x,
                                                    c->d_ge, c->d_He32, project, tscene, sproj);
}
void launch_gather_grad(ms_ctx* c, const double* x, double h2, double* g) {
  k_gather_grad<<<nblocks(c->n, 64), 64, 0, c->stream>>>(c->n, c->d_vt_ptr, c->d_vt_code, c->d_ge, c->d_mass, x,
                                                          c->d_xtilde, h2, c->gravity[0], c->gravity[1],
                                                          c->gravity[2], hs_of(c), g);
}
void launch_gather_hess(ms_ctx* c, const double* x, double h2, int prec) {
  const int S = c->pat.S;
  dim3 grid(unsigned(c->pat.nslices), unsigned((c->pat.maxw * S + 63) / 64));
  if (prec == MS_PREC_FP64)
    k_gather_hess<double, double><<<grid, 64, 0, c->stream>>>(c->n, S, c->pat.d_slice_base, c->pat.d_col, c->d_gptr,
                                                             c->d_gcode, c->d_He, c->d_mass, x, h2, hs_of(c),
                                                             c->d_vals);
  else
    k_gather_hess<float, float><<<grid, 64, 0, c->stream>>>(c->n, S, c->pat.d_slice_base, c->pat.d_col, c->d_gptr,
                                                           c->d_gcode, c->d_He32, c->d_mass, x, h2, hs_of(c),
                                                           c->d_vals32);
}
// vals[diag block of v] += sign * h^2 kappa b''(d_v) n n^T (the barrier
// curvature that the gather kernel adds on diagonal slots).
template <typename VT>
__global__ void k_diag_barrier(int64_t n, int S, const int32_t* __restrict__ diag_slot,
                               const double* __restrict__ x, const double* __restrict__ mass, HalfSpace hs,
                               double h2, double sign, VT* __restrict__ vals) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n || !(mass[v] > 0.0)) return;  // as the gather: no contact on massless vertices
  double b, b1, b2;
  barrier_terms(hs.n[0] * x[3 * v] + hs.n[1] * x[3 * v + 1] + hs.n[2] * x[3 * v + 2] - hs.off, hs.dhat, b, b1, b2);
  if (b2 == 0.0) return;
  const double f = sign * h2 * hs.kappa * b2;
  VT* out = vals + vbase(diag_slot[v], S);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) out[S * (3 * i + j)] = VT(double(out[S * (3 * i + j)]) + f * hs.n[i] * hs.n[j]);
}

void launch_diag_barrier(ms_ctx* c, int prec, void* vals, const double* x, double h2, double sign) {
  if (!c->has_hs) return;
  if (prec == MS_PREC_FP64)
    k_diag_barrier<double><<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, c->pat.S, c->pat.d_diag_slot, x, c->d_mass,
                                                                      hs_of(c), h2, sign, static_cast<double*>(vals));
  else
    k_diag_barrier<float><<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, c->pat.S, c->pat.d_diag_slot, x, c->d_mass,
                                                                     hs_of(c), h2, sign, static_cast<float*>(vals));
}

void launch_energy(ms_ctx* c, const double* x, const double* d, double alpha, double h2) {
  const int64_t m = std::max(c->T, c->n);
  k_energy<<<nblocks(m, 256), 256, 0, c->stream>>>(c->T, c->n, c->d_tets, c->d_Dminv, c->d_vol, c->d_mu, c->d_lam,
                                                  c->d_mass, x, d, alpha, c->d_xtilde, h2, c->gravity[0],
                                                  c->gravity[1], c->gravity[2], hs_of(c), c->d_part, c->d_counter,
                                                  c->d_scal + S_E0);
}
void launch_energy_delta(ms_ctx* c, const double* x, const double* d, double alpha, double h2) {
  const int64_t m = std::max(c->T, c->n);
  k_energy_delta<<<nblocks(m, 256), 256, 0, c->stream>>>(c->T, c->n, c->d_tets, c->d_Dminv, c->d_vol, c->d_mu,
                                                        c->d_lam, c->d_mass, x, d, alpha, c->d_xtilde, h2,
                                                        c->gravity[0], c->gravity[1], c->gravity[2], hs_of(c),
                                                        c->d_part, c->d_counter, c->d_scal + S_DE0);
}
void launch_ccd(ms_ctx* c, const double* x, const double* d) {
  k_ccd<<<nblocks(c->n, 256), 256, 0, c->stream>>>(c->n, x, d, hs_of(c), 0.9, c->d_part, c->d_counter,
                                                  c->d_scal + S_CCD);
}

}  // namespace ms
