// Dense FP64 inverse of the coarse operator U^T H U (symmetric positive
// definite up to null directions of U) by blocked Gauss-Jordan elimination
// without pivoting, in NB x NB tiles staged through LDS.  For an SPD matrix
// the eliminated pivot blocks are the Schur complements of a block Cholesky
// (LDL^T) factorisation, so no pivoting is needed; the explicit inverse is
// what the preconditioner applies every PCG iteration (one GEMV).
//
// Panel k (tile row/column k of the current matrix A):
//   k_gj_diag    D = inv(A_kk): in-place Gauss-Jordan of one tile by one
//                block; a pivot below 1e-12 of the original diagonal is
//                replaced by that diagonal (keeps the result SPD when U has
//                null directions, e.g. a handle with degenerate support)
//   k_gj_col     W_ik = A_ik D and V_kj = D A_kj for every i, j != k
//   k_gj_update  A_ij -= W_ik A_kj for i, j != k
//   k_gj_fix     A_ik = -W_ik, A_kj = V_kj, A_kk = D
// After the last panel A holds the inverse.  The matrix is padded to a
// multiple of NB with identity rows; the leading dimension is rp.
#include "ms_internal.h"

namespace ms {

constexpr int NB = 64;

__device__ __forceinline__ void load_tile(double (*s)[NB + 1], const double* __restrict__ A, int rp, int ti, int tj) {
  for (int q = threadIdx.x; q < NB * NB; q += blockDim.x) {
    const int a = q / NB, b = q % NB;
    s[a][b] = A[int64_t(ti * NB + a) * rp + tj * NB + b];
  }
}

// Gauss-Jordan inverse of tile (k,k) by one block of 256 threads: thread
// (a, b) keeps the 4 x 4 sub-block of rows 4a.. and columns 4b.. in
// registers.  At pivot P the owners of column P and of row P publish them in
// LDS; every thread then updates its entries with the same operations per
// entry as a column-by-column elimination.  A pivot below 1e-12 of the
// original diagonal is replaced by that diagonal.
__global__ void __launch_bounds__(256) k_gj_diag(int rp, int k, const double* __restrict__ A,
                                                 double* __restrict__ Dk, const double* __restrict__ diag0,
                                                 int* __restrict__ nreg) {
  __shared__ double s_col[NB], s_row[NB], s_d0[NB];
  const int t = threadIdx.x, a = t / 16, b = t % 16;
  double m[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) m[u][v] = A[int64_t(k * NB + 4 * a + u) * rp + k * NB + 4 * b + v];
  if (t < NB) s_d0[t] = diag0[k * NB + t];
  for (int P = 0; P < NB; ++P) {
    const int pq = P / 4, pr = P % 4;
    if (b == pq)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double v = m[u][0];
#pragma unroll
        for (int w = 1; w < 4; ++w)
          if (pr == w) v = m[u][w];
        s_col[4 * a + u] = v;
      }
    if (a == pq)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double x = m[0][v];
#pragma unroll
        for (int w = 1; w < 4; ++w)
          if (pr == w) x = m[w][v];
        s_row[4 * b + v] = x;
      }
    __syncthreads();
    double piv = s_col[P];
    const double d0 = s_d0[P];
    if (!(piv > 1e-12 * d0) || !isfinite(piv)) {
      piv = d0 > 0 ? d0 : 1.0;
      if (t == 0) atomicAdd(nreg, 1);
    }
    const double ip = 1.0 / piv;
    double fi[4], rowp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) fi[u] = s_col[4 * a + u];
#pragma unroll
    for (int v = 0; v < 4; ++v) rowp[v] = (4 * b + v == P) ? ip : s_row[4 * b + v] * ip;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * a + u, j = 4 * b + v;
        m[u][v] = (i == P) ? rowp[v] : ((j == P) ? -fi[u] * ip : m[u][v] - fi[u] * rowp[v]);
      }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) Dk[(4 * a + u) * NB + 4 * b + v] = m[u][v];
}

// 64 x 64 x 64 tile product from LDS: acc += A B (thread: 4 x 4 outputs).
__device__ __forceinline__ void tile_mma(const double (*sA)[NB + 1], const double (*sB)[NB + 1], double acc[4][4],
                                         int r0, int c0) {
  for (int l = 0; l < NB; ++l) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = sA[r0 + u][l];
      b[u] = sB[l][c0 + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
  }
}

// blockIdx.y = 0: W_ik = A_ik D_k for tile rows i != k; blockIdx.y = 1:
// V_ki = D_k A_ki for tile columns i != k (blockIdx.x enumerates i).
__global__ void __launch_bounds__(256) k_gj_col(int rp, int k, const double* __restrict__ A,
                                                const double* __restrict__ Dk, double* __restrict__ W,
                                                double* __restrict__ V) {
  __shared__ double sA[NB][NB + 1];
  __shared__ double sD[NB][NB + 1];
  const int i = int(blockIdx.x) < k ? int(blockIdx.x) : int(blockIdx.x) + 1;
  const bool row = blockIdx.y == 1;
  if (row)
    load_tile(sA, A, rp, k, i);
  else
    load_tile(sA, A, rp, i, k);
  for (int q = threadIdx.x; q < NB * NB; q += blockDim.x) sD[q / NB][q % NB] = Dk[q];
  __syncthreads();
  const int r0 = (threadIdx.x / 16) * 4, c0 = (threadIdx.x % 16) * 4;
  double acc[4][4] = {};
  if (row)
    tile_mma(sD, sA, acc, r0, c0);
  else
    tile_mma(sA, sD, acc, r0, c0);
  double* out = (row ? V : W) + int64_t(i) * NB * NB;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(r0 + u) * NB + c0 + v] = acc[u][v];
}

// A_ij -= W_ik A_kj for i, j != k; grid (nt-1) x (nt-1).
__global__ void __launch_bounds__(256) k_gj_update(int rp, int k, double* __restrict__ A,
                                                   const double* __restrict__ W) {
  __shared__ double sW[NB][NB + 1];
  __shared__ double sR[NB][NB + 1];
  const int i = int(blockIdx.y) < k ? int(blockIdx.y) : int(blockIdx.y) + 1;
  const int j = int(blockIdx.x) < k ? int(blockIdx.x) : int(blockIdx.x) + 1;
  for (int q = threadIdx.x; q < NB * NB; q += blockDim.x) sW[q / NB][q % NB] = W[int64_t(i) * NB * NB + q];
  load_tile(sR, A, rp, k, j);
  __syncthreads();
  const int r0 = (threadIdx.x / 16) * 4, c0 = (threadIdx.x % 16) * 4;
  double acc[4][4] = {};
  tile_mma(sW, sR, acc, r0, c0);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) A[int64_t(i * NB + r0 + u) * rp + j * NB + c0 + v] -= acc[u][v];
}

// Row and column k of the result: A_ik = -W_ik, A_ki = V_ki, A_kk = D.
__global__ void __launch_bounds__(256) k_gj_fix(int rp, int k, double* __restrict__ A, const double* __restrict__ W,
                                                const double* __restrict__ V, const double* __restrict__ Dk) {
  const int i = blockIdx.x;
  for (int q = threadIdx.x; q < NB * NB; q += blockDim.x) {
    const int a = q / NB, b = q % NB;
    if (i == k) {
      A[int64_t(k * NB + a) * rp + k * NB + b] = Dk[q];
    } else {
      A[int64_t(i * NB + a) * rp + k * NB + b] = -W[int64_t(i) * NB * NB + q];
      A[int64_t(k * NB + a) * rp + i * NB + b] = V[int64_t(i) * NB * NB + q];
    }
  }
}

// Largest diagonal entry of the r x r Galerkin matrix (one block).
__global__ void __launch_bounds__(256) k_diag_max(int r, const double* __restrict__ A, double* __restrict__ out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < r; i += blockDim.x) m = fmax(m, A[int64_t(i) * r + i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0] > 0 ? sh[0] : 1.0;
}

// Copy the r x r Galerkin matrix into the padded rp x rp workspace (identity
// padding) and record the diagonal used by the pivot safeguard; diagonal
// entries that are not positive (null directions of U) get the largest one.
__global__ void k_pad_copy(int r, int rp, const double* __restrict__ A, double* __restrict__ L,
                           double* __restrict__ diag0, const double* __restrict__ dmax_p) {
  const double dmax = dmax_p[0];
  for (int64_t q = threadIdx.x + int64_t(blockIdx.x) * blockDim.x; q < int64_t(rp) * rp;
       q += int64_t(blockDim.x) * gridDim.x) {
    const int i = int(q / rp), j = int(q % rp);
    double v;
    if (i < r && j < r) {
      v = A[int64_t(i) * r + j];
      if (i == j && !(v > 1e-14 * dmax)) v = dmax;
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    L[q] = v;
    if (i == j) diag0[i] = v;
  }
}

// FP32 copy of the inverse, symmetrised: out_ij = (A_ij + A_ji) / 2.
__global__ void k_inverse_f32(int rp, const double* __restrict__ A, float* __restrict__ out) {
  for (int64_t q = threadIdx.x + int64_t(blockIdx.x) * blockDim.x; q < int64_t(rp) * rp;
       q += int64_t(blockDim.x) * gridDim.x) {
    const int64_t i = q / rp, j = q % rp;
    out[q] = float(0.5 * (A[q] + A[j * rp + i]));
  }
}

ms_status coarse_factor(ms_ctx* c) {
  const int r = c->r, rp = c->rp, nt = rp / NB;
  MS_HIP(hipMemsetAsync(c->d_nreg, 0, sizeof(int), c->stream));
  k_diag_max<<<1, 256, 0, c->stream>>>(r, c->d_Ac, c->d_diag0 + rp);
  k_pad_copy<<<256, 256, 0, c->stream>>>(r, rp, c->d_Ac, c->d_Ainv, c->d_diag0, c->d_diag0 + rp);
  for (int k = 0; k < nt; ++k) {
    k_gj_diag<<<1, 256, 0, c->stream>>>(rp, k, c->d_Ainv, c->d_Linvd, c->d_diag0, c->d_nreg);
    if (nt > 1) {
      k_gj_col<<<dim3(unsigned(nt - 1), 2), 256, 0, c->stream>>>(rp, k, c->d_Ainv, c->d_Linvd, c->d_Y, c->d_Lc);
      k_gj_update<<<dim3(unsigned(nt - 1), unsigned(nt - 1)), 256, 0, c->stream>>>(rp, k, c->d_Ainv, c->d_Y);
    }
    k_gj_fix<<<unsigned(nt), 256, 0, c->stream>>>(rp, k, c->d_Ainv, c->d_Y, c->d_Lc, c->d_Linvd);
  }
  k_inverse_f32<<<1024, 256, 0, c->stream>>>(rp, c->d_Ainv, c->d_Ainv32);
  c->coarse_valid = 1;
  return MS_OK;
}

int coarse_pad(int r) { return ((r + NB - 1) / NB) * NB; }

}  // namespace ms
