// Learned coarse warm start (an addition to the paper's method): a
// three-layer perceptron with SiLU activations predicts the next coarse
// state q^{t+1} from (q^{t-1}, q^t) as a correction of the constant-velocity
// guess 2 q^t - q^{t-1}; the timestep then starts from
// x^t + U (q_hat - q^t) when that lowers the energy.
//
// Dense products run on the matrix cores: 64x64 output tiles per block of
// four waves, each wave a 32x32 quadrant of 2x2 MFMA 16x16x32 bf16 tiles
// (gfx950) with FP32 accumulation; operands are FP32 in memory and rounded to bf16
// (nearest even) as they are staged through LDS.  Training is Adam on FP32
// master weights over caller-given minibatches (deterministic: no atomics,
// fixed reduction orders).
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "ms_internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct Mlp {
  int in = 0, w = 0, out = 0;
  float* d_par = nullptr;  // W0 b0 W1 b1 W2 b2 contiguous (FP32; products round to bf16)
  float* d_mean = nullptr;
  float* d_std = nullptr;
  float* d_scale = nullptr;
  float* d_z = nullptr;    // [in] network input
  float* d_h = nullptr;    // [2 w + out] activations
  double* d_qprev = nullptr;
  double* d_qcur = nullptr;
};

namespace ms {

namespace {

__device__ __forceinline__ unsigned short to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  return static_cast<unsigned short>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// C[m][n] = sum_k opA[m][k] opB[k][n] (+ bias[n]) (+ C[m][n] if accumulate).
// TA: A stored [K][M] (else [M][K]); BNK: B stored [N][K] (else [K][N]).
// Each k-step stages a 64 x 32 slab of both operands in LDS as bf16 and
// feeds gfx950's 16x16x32 bf16 MFMA: lane l holds row (or column) l % 16 of
// its tile and the 8 consecutive k of group l / 16, one 16-byte LDS read.
template <bool TA, bool BNK>
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const float* __restrict__ A, int lda,
                                                   const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                   int ldc, const float* __restrict__ bias, int accumulate) {
  constexpr int KT = 32;   // k per step
  constexpr int LDK = 40;  // bf16 per LDS row (32 + 8: 80-byte rows keep the 16-byte reads aligned)
  __shared__ __align__(16) unsigned short As[64][LDK];
  __shared__ __align__(16) unsigned short Bs[64][LDK];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += KT) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = t + 256 * r;
      int mm, kk;
      if (TA) {
        kk = e / 64;
        mm = e % 64;
      } else {
        mm = e / KT;
        kk = e % KT;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      float va = 0.f;
      if (gm < M && gk < K) va = TA ? A[int64_t(gk) * lda + gm] : A[int64_t(gm) * lda + gk];
      As[mm][kk] = to_bf16(va);
      int nn;
      if (BNK) {
        nn = e / KT;
        kk = e % KT;
      } else {
        kk = e / 64;
        nn = e % 64;
      }
      const int gn = n0 + nn, gk2 = k0 + kk;
      float vb = 0.f;
      if (gn < N && gk2 < K) vb = BNK ? B[int64_t(gn) * ldb + gk2] : B[int64_t(gk2) * ldb + gn];
      Bs[nn][kk] = to_bf16(vb);
    }
    __syncthreads();
    v8bf a[2], b[2];
    const int kq = 8 * (lane >> 4), rr = lane & 15;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(&As[wm + 16 * i + rr][kq]));
      b[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(&Bs[wn + 16 * i + rr][kq]));
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // lane holds rows 4 (lane / 16) + q, column lane % 16 of each 16x16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + q, gn = n0 + wn + 16 * j + (lane & 15);
        if (gm < M && gn < N) {
          float v = acc[i][j][q];
          if (bias) v += bias[gn];
          float* cp = C + int64_t(gm) * ldc + gn;
          *cp = accumulate ? *cp + v : v;
        }
      }
}

__device__ __forceinline__ float silu_f(float x) { return x / (1.f + expf(-x)); }
__device__ __forceinline__ float silu_g(float x) {
  const float s = 1.f / (1.f + expf(-x));
  return s * (1.f + x * (1.f - s));
}

__global__ void k_silu(int64_t n, const float* __restrict__ h, float* __restrict__ a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = silu_f(h[i]);
}

__global__ void k_silu_back(int64_t n, const float* __restrict__ da, const float* __restrict__ h,
                            float* __restrict__ dh) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dh[i] = da[i] * silu_g(h[i]);
}

// dY = 2 (Y - T) / n and per-block partial sums of (Y - T)^2.
__global__ void __launch_bounds__(256) k_mse(int64_t n, const float* __restrict__ y, const float* __restrict__ tg,
                                             float* __restrict__ dy, double* __restrict__ part) {
  __shared__ double sh[256];
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    const float r = y[i] - tg[i];
    dy[i] = 2.f * r / float(n);
    e = double(r) * double(r);
  }
  sh[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// db[n] = sum over rows of dH[m][n] (rows in order).
__global__ void k_colsum(int M, int N, const float* __restrict__ dh, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += dh[int64_t(m) * N + j];
  db[j] = s;
}

__global__ void k_gather_rows(int B, int D, const int32_t* __restrict__ idx, const float* __restrict__ src,
                              float* __restrict__ dst) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(B) * D) return;
  const int b = int(e / D), d = int(e % D);
  dst[e] = src[int64_t(idx[b]) * D + d];
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

inline unsigned nb1(int64_t n) { return unsigned((n + 255) / 256); }

void gemm(hipStream_t st, bool ta, bool bnk, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
          float* C, int ldc, const float* bias, bool accumulate) {
  const dim3 grid(unsigned((N + 63) / 64), unsigned((M + 63) / 64));
  const int acc = accumulate ? 1 : 0;
  if (!ta && bnk)
    k_gemm_bf16<false, true><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, acc);
  else if (!ta && !bnk)
    k_gemm_bf16<false, false><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, acc);
  else if (ta && !bnk)
    k_gemm_bf16<true, false><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, acc);
  else
    k_gemm_bf16<true, true><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, acc);
}

struct Layout {
  int in, w, out;
  int64_t W0, b0, W1, b1, W2, b2, total;
  Layout(int i, int wd, int o) : in(i), w(wd), out(o) {
    W0 = 0;
    b0 = W0 + int64_t(w) * in;
    W1 = b0 + w;
    b1 = W1 + int64_t(w) * w;
    W2 = b1 + w;
    b2 = W2 + int64_t(out) * w;
    total = b2 + out;
  }
};

// Forward pass of a batch: Z [B][in] -> Y [B][out]; H0, H1 pre-activations
// and A0, A1 activations [B][w] kept for the backward pass.
void forward(hipStream_t st, const Layout& L, const float* par, int B, const float* Z, float* H0, float* A0,
             float* H1, float* A1, float* Y) {
  gemm(st, false, true, B, L.w, L.in, Z, L.in, par + L.W0, L.in, H0, L.w, par + L.b0, false);
  k_silu<<<nb1(int64_t(B) * L.w), 256, 0, st>>>(int64_t(B) * L.w, H0, A0);
  gemm(st, false, true, B, L.w, L.w, A0, L.w, par + L.W1, L.w, H1, L.w, par + L.b1, false);
  k_silu<<<nb1(int64_t(B) * L.w), 256, 0, st>>>(int64_t(B) * L.w, H1, A1);
  gemm(st, false, true, B, L.out, L.w, A1, L.w, par + L.W2, L.w, Y, L.out, par + L.b2, false);
}

struct DevBuf {
  const ms_device* dev;
  std::vector<void*> ptrs;
  explicit DevBuf(const ms_device* d) : dev(d) {}
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
  ~DevBuf() {
    for (void* p : ptrs) {
      if (dev->free)
        dev->free(p, dev->user);
      else
        (void)hipFree(p);
    }
  }
};

}  // namespace

void destroy_mlp(ms_ctx* c) {
  delete c->mlp;  // device buffers belong to the context's allocation list
  c->mlp = nullptr;
}

// Learned warm start, called at step start with x = x^t (Dirichlet
// applied); falls back to the inertial predictor (if enabled) while no
// prediction is available.
ms_status warm_start(ms_ctx* c, double dt, bool inertial, int32_t* used) {
  *used = 0;
  Mlp* N = c->mlp;
  if (!N || !c->has_basis || c->q_hist < 2) return inertial ? inertial_start(c, dt * dt) : MS_OK;
  const int r = c->r;
  // z = ([q^{t-1}, q^t] - mean) / std, then the network, then
  // dq = (q^t - q^{t-1}) + out_scale * y  (= q_hat - q^t)
  std::vector<double> qp(r), qc(r);
  MS_HIP(hipMemcpyAsync(qp.data(), N->d_qprev, r * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  MS_HIP(hipMemcpyAsync(qc.data(), N->d_qcur, r * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  std::vector<float> mean(N->in), sd(N->in), scale(N->out);
  MS_HIP(hipMemcpyAsync(mean.data(), N->d_mean, N->in * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  MS_HIP(hipMemcpyAsync(sd.data(), N->d_std, N->in * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  MS_HIP(hipMemcpyAsync(scale.data(), N->d_scale, N->out * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  ms_status s = sync(c);
  if (s) return s;
  std::vector<float> z(N->in);
  for (int i = 0; i < r; ++i) {
    z[i] = float((qp[i] - mean[i]) / sd[i]);
    z[r + i] = float((qc[i] - mean[r + i]) / sd[r + i]);
  }
  MS_HIP(hipMemcpyAsync(N->d_z, z.data(), N->in * sizeof(float), hipMemcpyHostToDevice, c->stream));
  const Layout L(N->in, N->w, N->out);
  float* H0 = N->d_h;
  float* A0 = H0 + N->w;
  float* H1 = A0 + N->w;
  float* A1 = H1 + N->w;
  float* Y = A1 + N->w;
  forward(c->stream, L, N->d_par, 1, N->d_z, H0, A0, H1, A1, Y);
  std::vector<float> y(N->out);
  MS_HIP(hipMemcpyAsync(y.data(), Y, N->out * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  if ((s = sync(c))) return s;
  // the network's correction of the constant-velocity coarse guess; the
  // inertial predictor's coarse part is exactly that guess (q is linear in
  // x and x~ = 2 x^t - x^{t-1}), so with the predictor on, the learned start
  // is x~ + U (out_scale * y), else x^t + U (q^t - q^{t-1} + out_scale * y)
  std::vector<double> dq(r);
  for (int i = 0; i < r; ++i) {
    dq[i] = double(scale[i]) * double(y[i]) + (inertial ? 0.0 : qc[i] - qp[i]);
    if (!std::isfinite(dq[i])) return inertial ? inertial_start(c, dt * dt) : MS_OK;  // no usable prediction
  }
  MS_HIP(hipMemcpyAsync(c->d_e, dq.data(), r * sizeof(double), hipMemcpyHostToDevice, c->stream));
  const double h2 = dt * dt;
  auto candidate = [&](double* dE, double* alpha) -> ms_status {
    *alpha = 1.0;
    ms_status st;
    if (c->has_hs) {
      launch_ccd(c, c->d_x, c->d_d);
      if ((st = read_scal(c))) return st;
      *alpha = std::fmin(1.0, c->h_scal[S_CCD]);
    }
    double err;
    return energy_delta(c, c->d_x, c->d_d, *alpha, h2, dE, &err);
  };
  // candidates: the inertial predictor x~ (if on) and x~ + beta U dq for
  // beta = 1, 1/2, 1/4 (from x^t without the predictor); the lowest-energy
  // one is taken if it lowers E
  const size_t nb = 3 * c->n * sizeof(double);
  double best = INFINITY, best_a = 0.0, best_beta = -1.0;
  if (inertial) {
    launch_predictor_dir(c);  // x~ - x, zero on pinned vertices
    double dE_i, a_i;
    if ((s = candidate(&dE_i, &a_i))) return s;
    if (std::isfinite(dE_i) && dE_i < 0.0) best = dE_i, best_a = a_i, best_beta = 0.0;
    MS_HIP(hipMemcpyAsync(c->d_p, c->d_d, nb, hipMemcpyDeviceToDevice, c->stream));
  } else {
    launch_fill(c, c->d_p, 0.0, 3 * c->n);
  }
  launch_prolong_set_d(c);  // U dq (zero on pinned vertices), kept in w
  MS_HIP(hipMemcpyAsync(c->d_w, c->d_d, nb, hipMemcpyDeviceToDevice, c->stream));
  for (const double beta : {1.0, 0.5, 0.25}) {
    MS_HIP(hipMemcpyAsync(c->d_d, c->d_p, nb, hipMemcpyDeviceToDevice, c->stream));
    launch_axpy(c, c->d_d, c->d_w, beta, 3 * c->n);
    double dE_l, a_l;
    if ((s = candidate(&dE_l, &a_l))) return s;
    if (std::isfinite(dE_l) && dE_l < 0.0 && dE_l < best) best = dE_l, best_a = a_l, best_beta = beta;
  }
  if (best_beta < 0.0) return MS_OK;  // no candidate lowers E: start at x^t
  MS_HIP(hipMemcpyAsync(c->d_d, c->d_p, nb, hipMemcpyDeviceToDevice, c->stream));
  if (best_beta > 0.0) {
    launch_axpy(c, c->d_d, c->d_w, best_beta, 3 * c->n);
    *used = 1;
  }
  launch_axpy(c, c->d_x, c->d_d, best_a, 3 * c->n);
  return MS_OK;
}

// After a converged step: shift the coarse history.
ms_status record_coarse(ms_ctx* c) {
  Mlp* N = c->mlp;
  if (!N) return MS_OK;
  // q(x^{t+1}) (and, on the first record, q(x^t)) go to scratch first, so
  // that a failure leaves the history as it was
  ms_status s = coarse_coordinates(c, c->d_x, nullptr, c->d_e);
  if (s) return s;
  if (c->q_hist == 0 && (s = coarse_coordinates(c, c->d_xt, nullptr, c->d_c))) return s;
  std::swap(N->d_qprev, N->d_qcur);
  MS_HIP(hipMemcpyAsync(N->d_qcur, c->d_e, c->r * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (c->q_hist == 0) {
    MS_HIP(hipMemcpyAsync(N->d_qprev, c->d_c, c->r * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    c->q_hist = 1;
  }
  ++c->q_hist;
  return MS_OK;
}

}  // namespace ms

using namespace ms;

extern "C" {

ms_status ms_set_warmstart(ms_ctx* c, const ms_mlp_desc* d) {
  if (!c) return MS_E_ARG;
  if (!c->has_basis) return fail(c, MS_E_ORDER, "the warm start needs a basis");
  if (!d) {  // remove
    destroy_mlp(c);
    return MS_OK;
  }
  const int r = c->r;
  if (d->in_dim != 2 * r || d->out_dim != r || d->width < 1 || !d->W0 || !d->b0 || !d->W1 || !d->b1 || !d->W2 ||
      !d->b2 || !d->in_mean || !d->in_std || !d->out_scale)
    return fail(c, MS_E_ARG, "network shape must be 2r -> width -> width -> r with r = 12 m");
  const Layout L(d->in_dim, d->width, d->out_dim);
  std::vector<float> par(L.total);
  std::memcpy(&par[L.W0], d->W0, sizeof(float) * L.w * L.in);
  std::memcpy(&par[L.b0], d->b0, sizeof(float) * L.w);
  std::memcpy(&par[L.W1], d->W1, sizeof(float) * L.w * L.w);
  std::memcpy(&par[L.b1], d->b1, sizeof(float) * L.w);
  std::memcpy(&par[L.W2], d->W2, sizeof(float) * L.out * L.w);
  std::memcpy(&par[L.b2], d->b2, sizeof(float) * L.out);
  for (float v : par)
    if (!std::isfinite(v)) return fail(c, MS_E_NONFINITE, "non-finite network weight");
  for (int i = 0; i < L.in; ++i)
    if (!(d->in_std[i] > 0.f)) return fail(c, MS_E_ARG, "input standard deviations must be positive");
  static_assert(sizeof(Mlp) > 0, "");
  if (!c->mlp) c->mlp = new Mlp();  // freed with the context (plain struct of device pointers)
  Mlp* N = c->mlp;
  N->in = L.in;
  N->w = L.w;
  N->out = L.out;
  ms_status s;
  if ((s = upload(c, &N->d_par, par.data(), par.size())) || (s = upload(c, &N->d_mean, d->in_mean, size_t(L.in))) ||
      (s = upload(c, &N->d_std, d->in_std, size_t(L.in))) ||
      (s = upload(c, &N->d_scale, d->out_scale, size_t(L.out))) || (s = alloc_n(c, &N->d_z, size_t(L.in))) ||
      (s = alloc_n(c, &N->d_h, size_t(4 * L.w + L.out))) || (s = alloc_n(c, &N->d_qprev, size_t(r))) ||
      (s = alloc_n(c, &N->d_qcur, size_t(r))))
    return s;
  c->q_hist = 0;
  return MS_OK;
}

ms_status ms_mlp_forward(const ms_device* dev, int32_t in_dim, int32_t width, int32_t out_dim, const float* params,
                         int64_t n, const float* Z, float* Y) {
  if (!dev || !params || !Z || !Y || in_dim < 1 || width < 1 || out_dim < 1 || n < 1) return MS_E_ARG;
  if (hipSetDevice(dev->device) != hipSuccess) return MS_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(dev->hip_stream);
  const Layout L(in_dim, width, out_dim);
  DevBuf buf(dev);
  float* par = buf.get<float>(L.total);
  float* z = buf.get<float>(size_t(n) * in_dim);
  float* h = buf.get<float>(size_t(n) * (4 * width + out_dim));
  if (!par || !z || !h) return MS_E_NOMEM;
  if (hipMemcpyAsync(par, params, L.total * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(z, Z, size_t(n) * in_dim * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
    return MS_E_DEVICE;
  float* H0 = h;
  float* A0 = H0 + n * width;
  float* H1 = A0 + n * width;
  float* A1 = H1 + n * width;
  float* Yd = A1 + n * width;
  forward(st, L, par, int(n), z, H0, A0, H1, A1, Yd);
  if (hipMemcpyAsync(Y, Yd, size_t(n) * out_dim * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return MS_E_DEVICE;
  return MS_OK;
}

}  // extern "C"

// ---- forward pass without allocation -------------------------------------
// Activation scratch of ms_mlp_forward_noalloc: a file-scope device array of
// MS_MLP_NOALLOC_SCRATCH_FLOATS floats.  Every GPU the library runs on holds
// its own copy until the process ends.  In host code the array's name is
// only a stand-in: kernels receive the device address taken per device by
// hipGetSymbolAddress (with that device current).
static __device__ __align__(256) float scratch[MS_MLP_NOALLOC_SCRATCH_FLOATS];

namespace {
std::mutex g_scratch_mu;
std::vector<float*> g_scratch_ptr;  // per device id

ms_status scratch_address(int device, float** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) return MS_E_ARG;
  if (int(g_scratch_ptr.size()) <= device) g_scratch_ptr.resize(size_t(device) + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MS_E_DEVICE;
    g_scratch_ptr[device] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[device];
  return MS_OK;
}
}  // namespace

extern "C" {

ms_status ms_mlp_forward_noalloc(const ms_device* dev, int32_t in_dim, int32_t width, int32_t out_dim,
                                 const float* params, int64_t n, const float* Z, float* Y) {
  if (!dev || !params || !Z || !Y || in_dim < 1 || width < 1 || out_dim < 1 || n < 1) return MS_E_ARG;
  // activations H0, A0, H1, A1: 4 n width floats
  if (n > int64_t(MS_MLP_NOALLOC_SCRATCH_FLOATS) / (4 * int64_t(width))) return MS_E_ARG;
  if (hipSetDevice(dev->device) != hipSuccess) return MS_E_DEVICE;
  float* h = nullptr;
  const ms_status s = scratch_address(dev->device, &h);
  if (s) return s;
  hipStream_t st = static_cast<hipStream_t>(dev->hip_stream);
  const Layout L(in_dim, width, out_dim);
  float* H0 = h;
  float* A0 = H0 + n * width;
  float* H1 = A0 + n * width;
  float* A1 = H1 + n * width;
  // every activation is written before it is read: nothing to clear
  forward(st, L, params, int(n), Z, H0, A0, H1, A1, Y);
  return hipGetLastError() == hipSuccess ? MS_OK : MS_E_DEVICE;
}

ms_status ms_mlp_train(const ms_device* dev, int32_t in_dim, int32_t width, int32_t out_dim, float* params,
                       int64_t n_samples, const float* X, const float* T, int32_t n_steps, int32_t batch,
                       const int32_t* order, float lr, float* losses, float* first_grads) {
  if (!dev || !params || !X || !T || !order || in_dim < 1 || width < 1 || out_dim < 1 || n_samples < 1 ||
      n_steps < 1 || batch < 1 || !(lr > 0.f))
    return MS_E_ARG;
  for (int64_t i = 0; i < int64_t(n_steps) * batch; ++i)
    if (order[i] < 0 || order[i] >= n_samples) return MS_E_ARG;
  if (hipSetDevice(dev->device) != hipSuccess) return MS_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(dev->hip_stream);
  const Layout L(in_dim, width, out_dim);
  const int B = batch, w = width;
  DevBuf buf(dev);
  float* par = buf.get<float>(L.total);
  float* grad = buf.get<float>(L.total);
  float* mom = buf.get<float>(L.total);
  float* vel = buf.get<float>(L.total);
  float* Xd = buf.get<float>(size_t(n_samples) * in_dim);
  float* Td = buf.get<float>(size_t(n_samples) * out_dim);
  int32_t* ord = buf.get<int32_t>(size_t(n_steps) * B);
  float* Z = buf.get<float>(size_t(B) * in_dim);
  float* Tb = buf.get<float>(size_t(B) * out_dim);
  float* H0 = buf.get<float>(size_t(B) * w);
  float* A0 = buf.get<float>(size_t(B) * w);
  float* H1 = buf.get<float>(size_t(B) * w);
  float* A1 = buf.get<float>(size_t(B) * w);
  float* Y = buf.get<float>(size_t(B) * out_dim);
  float* dY = buf.get<float>(size_t(B) * out_dim);
  float* dA = buf.get<float>(size_t(B) * w);
  float* dH = buf.get<float>(size_t(B) * w);
  const int64_t nloss = (int64_t(B) * out_dim + 255) / 256;
  double* lpart = buf.get<double>(size_t(nloss) * n_steps);
  if (!par || !grad || !mom || !vel || !Xd || !Td || !ord || !Z || !Tb || !H0 || !A0 || !H1 || !A1 || !Y || !dY ||
      !dA || !dH || !lpart)
    return MS_E_NOMEM;
  auto H2D = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  if (!H2D(par, params, L.total * sizeof(float)) || !H2D(Xd, X, size_t(n_samples) * in_dim * sizeof(float)) ||
      !H2D(Td, T, size_t(n_samples) * out_dim * sizeof(float)) ||
      !H2D(ord, order, size_t(n_steps) * B * sizeof(int32_t)) ||
      hipMemsetAsync(mom, 0, L.total * sizeof(float), st) != hipSuccess ||
      hipMemsetAsync(vel, 0, L.total * sizeof(float), st) != hipSuccess)
    return MS_E_DEVICE;
  double c1 = 1.0, c2 = 1.0;
  for (int s = 0; s < n_steps; ++s) {
    const int32_t* idx = ord + int64_t(s) * B;
    k_gather_rows<<<nb1(int64_t(B) * in_dim), 256, 0, st>>>(B, in_dim, idx, Xd, Z);
    k_gather_rows<<<nb1(int64_t(B) * out_dim), 256, 0, st>>>(B, out_dim, idx, Td, Tb);
    forward(st, L, par, B, Z, H0, A0, H1, A1, Y);
    k_mse<<<unsigned(nloss), 256, 0, st>>>(int64_t(B) * out_dim, Y, Tb, dY, lpart + int64_t(s) * nloss);
    // layer 2: dW2 = dY^T A1, db2, dA1 = dY W2
    gemm(st, true, false, out_dim, w, B, dY, out_dim, A1, w, grad + L.W2, w, nullptr, false);
    k_colsum<<<nb1(out_dim), 256, 0, st>>>(B, out_dim, dY, grad + L.b2);
    gemm(st, false, false, B, w, out_dim, dY, out_dim, par + L.W2, w, dA, w, nullptr, false);
    k_silu_back<<<nb1(int64_t(B) * w), 256, 0, st>>>(int64_t(B) * w, dA, H1, dH);
    // layer 1
    gemm(st, true, false, w, w, B, dH, w, A0, w, grad + L.W1, w, nullptr, false);
    k_colsum<<<nb1(w), 256, 0, st>>>(B, w, dH, grad + L.b1);
    gemm(st, false, false, B, w, w, dH, w, par + L.W1, w, dA, w, nullptr, false);
    k_silu_back<<<nb1(int64_t(B) * w), 256, 0, st>>>(int64_t(B) * w, dA, H0, dH);
    // layer 0
    gemm(st, true, false, w, in_dim, B, dH, w, Z, in_dim, grad + L.W0, in_dim, nullptr, false);
    k_colsum<<<nb1(w), 256, 0, st>>>(B, w, dH, grad + L.b0);
    if (s == 0 && first_grads)
      if (hipMemcpyAsync(first_grads, grad, L.total * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess)
        return MS_E_DEVICE;
    c1 *= 0.9;
    c2 *= 0.999;
    k_adam<<<nb1(L.total), 256, 0, st>>>(L.total, par, grad, mom, vel, lr, float(1.0 - c1), float(1.0 - c2));
  }
  std::vector<double> lp(size_t(nloss) * n_steps);
  if (hipMemcpyAsync(lp.data(), lpart, lp.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(params, par, L.total * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return MS_E_DEVICE;
  if (losses)
    for (int s = 0; s < n_steps; ++s) {
      double sum = 0.0;
      for (int64_t b = 0; b < nloss; ++b) sum += lp[size_t(s) * nloss + b];
      losses[s] = float(sum / (double(B) * out_dim));
    }
  return MS_OK;
}

}  // extern "C"
