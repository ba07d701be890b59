// Dense FP64 solve of a symmetric positive definite system on the GPU, for
// the basis build's local biharmonic problems (Sec. 3.5): the sparse matrix
// (full symmetric CSR) is scattered into a dense lower triangle padded to a
// multiple of NB with identity rows, factored by a right-looking blocked
// Cholesky in NB x NB tiles, and the right-hand side is solved by blocked
// forward and back substitution.
//
// Panel k:
//   k_chol_diag    L_kk = chol(A_kk) in LDS by one block, and its inverse
//                  (forward substitution per column); a pivot that is not
//                  positive sets the failure flag (the caller falls back)
//   k_chol_trsm    L_ik = A_ik L_kk^-T for every tile row i > k
//   k_chol_update  A_ij -= L_ik L_jk^T for k < j <= i
// Solve: y_k = L_kk^-1 b_k, b_i -= L_ik y_k (i > k), forward; then
// x_k = L_kk^-T y_k, y_j -= L_kj^T x_k (j < k), backward.
#include "ms_internal.h"

namespace ms {

namespace {

constexpr int NB = 64;

__device__ __forceinline__ void tile_load(double (*s)[NB + 1], const double* __restrict__ A, int64_t ld, int ti,
                                          int tj, bool transpose) {
  for (int q = threadIdx.x; q < NB * NB; q += blockDim.x) {
    const int a = q / NB, b = q % NB;
    const double v = A[int64_t(ti * NB + a) * ld + tj * NB + b];
    if (transpose)
      s[b][a] = v;
    else
      s[a][b] = v;
  }
}

// acc += X Y for 64 x 64 LDS tiles (thread: rows r0.., columns c0.., 4 x 4)
__device__ __forceinline__ void tile_mul(const double (*X)[NB + 1], const double (*Y)[NB + 1], double acc[4][4],
                                         int r0, int c0) {
  for (int l = 0; l < NB; ++l) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = X[r0 + u][l];
      b[u] = Y[l][c0 + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
  }
}

__global__ void k_dense_fill(int n, int64_t np, double* __restrict__ A) {
  for (int64_t q = threadIdx.x + int64_t(blockIdx.x) * blockDim.x; q < np * np; q += int64_t(blockDim.x) * gridDim.x) {
    const int64_t i = q / np, j = q % np;
    A[q] = (i == j && i >= n) ? 1.0 : 0.0;
  }
}

// lower triangle of the symmetric CSR matrix into A
__global__ void k_dense_scatter(int n, const int* __restrict__ ptr, const int* __restrict__ idx,
                                const double* __restrict__ val, int64_t np, double* __restrict__ A) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k)
    if (idx[k] <= i) A[int64_t(i) * np + idx[k]] = val[k];
}

__global__ void __launch_bounds__(256) k_chol_diag(int64_t np, int k, double* __restrict__ A, double* __restrict__ D,
                                                   int* __restrict__ flag) {
  __shared__ double s[NB][NB + 1];
  __shared__ double t[NB][NB + 1];
  const int tid = threadIdx.x;
  tile_load(s, A, np, k, k, false);
  __syncthreads();
  for (int p = 0; p < NB; ++p) {
    if (tid == 0) {
      double d = s[p][p];
      if (!(d > 0.0) || !isfinite(d)) {
        atomicOr(flag, 1);
        d = 1.0;
      }
      s[p][p] = sqrt(d);
    }
    __syncthreads();
    if (tid > p && tid < NB) s[tid][p] /= s[p][p];
    __syncthreads();
    for (int q = tid; q < NB * NB; q += blockDim.x) {
      const int i = q / NB, j = q % NB;
      if (j > p && j <= i) s[i][j] -= s[i][p] * s[j][p];
    }
    __syncthreads();
  }
  // inverse of the lower triangular factor, one column per thread
  if (tid < NB) {
    const int j = tid;
    for (int i = 0; i < NB; ++i) {
      if (i < j) {
        t[i][j] = 0.0;
        continue;
      }
      double acc = (i == j) ? 1.0 : 0.0;
      for (int l = j; l < i; ++l) acc -= s[i][l] * t[l][j];
      t[i][j] = acc / s[i][i];
    }
  }
  __syncthreads();
  for (int q = tid; q < NB * NB; q += blockDim.x) {
    const int i = q / NB, j = q % NB;
    A[int64_t(k * NB + i) * np + k * NB + j] = j <= i ? s[i][j] : 0.0;
    D[int64_t(k) * NB * NB + q] = t[i][j];
  }
}

__global__ void __launch_bounds__(256) k_chol_trsm(int64_t np, int k, double* __restrict__ A,
                                                   const double* __restrict__ D) {
  __shared__ double sa[NB][NB + 1];
  __shared__ double sb[NB][NB + 1];
  const int i = k + 1 + int(blockIdx.x);
  tile_load(sa, A, np, i, k, false);
  for (int q = threadIdx.x; q < NB * NB; q += blockDim.x) sb[q % NB][q / NB] = D[int64_t(k) * NB * NB + q];
  __syncthreads();
  const int r0 = (threadIdx.x / 16) * 4, c0 = (threadIdx.x % 16) * 4;
  double acc[4][4] = {};
  tile_mul(sa, sb, acc, r0, c0);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) A[int64_t(i * NB + r0 + u) * np + k * NB + c0 + v] = acc[u][v];
}

__global__ void __launch_bounds__(256) k_chol_update(int64_t np, int k, double* __restrict__ A) {
  const int i = k + 1 + int(blockIdx.y), j = k + 1 + int(blockIdx.x);
  if (j > i) return;
  __shared__ double sa[NB][NB + 1];
  __shared__ double sb[NB][NB + 1];
  tile_load(sa, A, np, i, k, false);
  tile_load(sb, A, np, j, k, true);
  __syncthreads();
  const int r0 = (threadIdx.x / 16) * 4, c0 = (threadIdx.x % 16) * 4;
  double acc[4][4] = {};
  tile_mul(sa, sb, acc, r0, c0);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) A[int64_t(i * NB + r0 + u) * np + j * NB + c0 + v] -= acc[u][v];
}

// b_k <- D_k b_k (trans: D_k^T b_k), one block of NB threads
__global__ void k_tri_diag(int k, const double* __restrict__ D, double* __restrict__ b, int trans) {
  __shared__ double sb[NB];
  const int r = threadIdx.x;
  sb[r] = b[k * NB + r];
  __syncthreads();
  const double* Dk = D + int64_t(k) * NB * NB;
  double acc = 0.0;
  for (int l = 0; l < NB; ++l) acc += (trans ? Dk[l * NB + r] : Dk[r * NB + l]) * sb[l];
  b[k * NB + r] = acc;
}

// forward: b_i -= L_ik b_k for i = k + 1 + blockIdx.x; backward (trans):
// b_j -= L_kj^T b_k for j = blockIdx.x < k
__global__ void k_tri_update(int64_t np, int k, const double* __restrict__ A, double* __restrict__ b, int trans) {
  __shared__ double sb[NB];
  const int r = threadIdx.x;
  sb[r] = b[k * NB + r];
  __syncthreads();
  double acc = 0.0;
  if (!trans) {
    const int i = k + 1 + int(blockIdx.x);
    const double* Lr = A + int64_t(i * NB + r) * np + k * NB;
    for (int l = 0; l < NB; ++l) acc += Lr[l] * sb[l];
    b[i * NB + r] -= acc;
  } else {
    const int j = int(blockIdx.x);
    for (int l = 0; l < NB; ++l) acc += A[int64_t(k * NB + l) * np + j * NB + r] * sb[l];
    b[j * NB + r] -= acc;
  }
}

}  // namespace

ms_status dense_spd_solve(ms_ctx* c, int n, const int* ptr, const int* idx, const double* val, double* rhs,
                          bool* ok) {
  *ok = false;
  if (hipSetDevice(c->dev.device) != hipSuccess) return MS_E_DEVICE;  // callers may be worker threads
  const int nt = (n + NB - 1) / NB;
  const int64_t np = int64_t(nt) * NB, nnz = ptr[n];
  double *A = nullptr, *D = nullptr, *b = nullptr, *v = nullptr;
  int *p = nullptr, *ix = nullptr, *flag = nullptr;
  ms_status s = MS_OK;
  auto release = [&]() {
    (void)hipStreamSynchronize(c->stream);
    for (void* q : {(void*)A, (void*)D, (void*)b, (void*)v, (void*)p, (void*)ix, (void*)flag})
      if (q) dfree(c, q);
  };
  if ((s = alloc_n(c, &A, size_t(np * np))) || (s = alloc_n(c, &D, size_t(nt) * NB * NB)) ||
      (s = alloc_n(c, &b, size_t(np))) || (s = alloc_n(c, &v, size_t(std::max<int64_t>(nnz, 1)))) ||
      (s = alloc_n(c, &p, size_t(n + 1))) || (s = alloc_n(c, &ix, size_t(std::max<int64_t>(nnz, 1)))) ||
      (s = alloc_n(c, &flag, 1))) {
    release();
    return s;
  }
  hipError_t e = hipSuccess;
  auto hip = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  hip(hipMemcpyAsync(p, ptr, (n + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
  hip(hipMemcpyAsync(ix, idx, nnz * sizeof(int), hipMemcpyHostToDevice, c->stream));
  hip(hipMemcpyAsync(v, val, nnz * sizeof(double), hipMemcpyHostToDevice, c->stream));
  hip(hipMemsetAsync(b, 0, np * sizeof(double), c->stream));
  hip(hipMemcpyAsync(b, rhs, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  hip(hipMemsetAsync(flag, 0, sizeof(int), c->stream));
  k_dense_fill<<<2048, 256, 0, c->stream>>>(n, np, A);
  k_dense_scatter<<<unsigned((n + 255) / 256), 256, 0, c->stream>>>(n, p, ix, v, np, A);
  for (int k = 0; k < nt; ++k) {
    k_chol_diag<<<1, 256, 0, c->stream>>>(np, k, A, D, flag);
    const int rem = nt - k - 1;
    if (rem > 0) {
      k_chol_trsm<<<unsigned(rem), 256, 0, c->stream>>>(np, k, A, D);
      k_chol_update<<<dim3(unsigned(rem), unsigned(rem)), 256, 0, c->stream>>>(np, k, A);
    }
  }
  for (int k = 0; k < nt; ++k) {
    k_tri_diag<<<1, NB, 0, c->stream>>>(k, D, b, 0);
    if (nt - k - 1 > 0) k_tri_update<<<unsigned(nt - k - 1), NB, 0, c->stream>>>(np, k, A, b, 0);
  }
  for (int k = nt - 1; k >= 0; --k) {
    k_tri_diag<<<1, NB, 0, c->stream>>>(k, D, b, 1);
    if (k > 0) k_tri_update<<<unsigned(k), NB, 0, c->stream>>>(np, k, A, b, 1);
  }
  int hflag = 1;
  hip(hipGetLastError());
  hip(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  hip(hipMemcpyAsync(rhs, b, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  hip(hipStreamSynchronize(c->stream));
  release();
  if (e != hipSuccess) return MS_E_DEVICE;
  *ok = hflag == 0;
  return MS_OK;
}

}  // namespace ms
