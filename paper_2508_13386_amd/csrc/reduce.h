// Deterministic reductions for wave64 hardware.
//
// Each block reduces its values with cross-lane shuffles and LDS, writes one
// partial per block, and the last block to arrive (integer counter) sums the
// partials in block order.  The summation order is fixed by the launch
// shape, so results are bitwise reproducible run to run; no floating-point
// atomics are used.
#pragma once
#include <hip/hip_runtime.h>

namespace ms {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ void store_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_coherent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide sum of NV values (blockDim.x a multiple of 64, at most 1024).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double sh[NV][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (nw == 1) return;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[i][wave] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[i][w];
    v[i] = s;
  }
  __syncthreads();
}

// Writes this block's partial sums and returns true in the last block to
// finish, where v then holds the grid-wide totals (in every thread).
template <int NV>
__device__ __forceinline__ bool grid_sum(double (&v)[NV], double* part, unsigned* counter) {
  __shared__ int last;
  block_sum<NV>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) store_coherent(&part[blockIdx.x * NV + i], v[i]);
    __threadfence();
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += load_coherent(&part[b * NV + i]);
  block_sum<NV>(acc);
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = acc[i];
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

}  // namespace ms
