// Multi-source geodesic Voronoi on the GPU for the basis build's K-means
// (Sec. 3.6): every vertex takes the nearest seed under the stiffness-
// weighted edge costs, ties to the lower seed index.  Jacobi sweeps: each
// vertex replaces (distance, label) by the lexicographic minimum of its own
// and of (d_v + cost, label_v) over its neighbours v, until a sweep changes
// nothing.  With positive costs the fixed point is the one multi-source
// Dijkstra reaches (each vertex's value is the minimum over its neighbours'
// final values plus the edge cost, compared the same way), so the labels
// and distances equal the host's bit for bit.
#include <limits>
#include <vector>

#include "ms_internal.h"

namespace ms {

namespace {

__global__ void __launch_bounds__(256) k_vor_init(int n, const int* __restrict__ seeds, int ns,
                                                  double* __restrict__ d, int* __restrict__ l) {
  const int v = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v < n) {
    d[v] = INFINITY;
    l[v] = -1;
  }
}

__global__ void k_vor_seeds(const int* __restrict__ seeds, int ns, double* __restrict__ d, int* __restrict__ l) {
  const int s = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s < ns) {  // later duplicates of a vertex win, as in the host's seeding loop
    d[seeds[s]] = 0.0;
    atomicMax(&l[seeds[s]], s);
  }
}

__global__ void __launch_bounds__(256) k_vor_sweep(int n, const int* __restrict__ ptr, const int* __restrict__ idx,
                                                   const double* __restrict__ cost, const double* __restrict__ d_in,
                                                   const int* __restrict__ l_in, double* __restrict__ d_out,
                                                   int* __restrict__ l_out, int* __restrict__ changed) {
  const int w = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= n) return;
  double bd = d_in[w];
  int bl = l_in[w];
  for (int k = ptr[w]; k < ptr[w + 1]; ++k) {
    const int v = idx[k];
    const int lv = l_in[v];
    if (lv < 0) continue;
    const double cand = d_in[v] + cost[k];
    if (cand < bd || (cand == bd && lv < bl)) {
      bd = cand;
      bl = lv;
    }
  }
  d_out[w] = bd;
  l_out[w] = bl;
  if (bd != d_in[w] || bl != l_in[w]) *changed = 1;
}

}  // namespace

ms_status DevGraph::upload(ms_ctx* c, const std::vector<int>& p, const std::vector<int>& ix,
                           const std::vector<double>& cost) {
  n = int(p.size()) - 1;
  ms_status s;
  if ((s = ms::upload(c, &ptr, p.data(), p.size())) || (s = ms::upload(c, &idx, ix.data(), ix.size())) ||
      (s = ms::upload(c, &len, cost.data(), cost.size())) || (s = alloc_n(c, &d[0], size_t(n))) ||
      (s = alloc_n(c, &d[1], size_t(n))) || (s = alloc_n(c, &l[0], size_t(n))) || (s = alloc_n(c, &l[1], size_t(n))) ||
      (s = alloc_n(c, &flags, size_t(kSweepChunk))) || (s = alloc_n(c, &seeds, size_t(n))))
    return s;
  return MS_OK;
}

void DevGraph::release(ms_ctx* c) {
  (void)hipStreamSynchronize(c->stream);
  for (void* q : {(void*)ptr, (void*)idx, (void*)len, (void*)d[0], (void*)d[1], (void*)l[0], (void*)l[1],
                  (void*)flags, (void*)seeds})
    if (q) dfree(c, q);
  ptr = idx = nullptr;
  len = nullptr;
  d[0] = d[1] = nullptr;
  l[0] = l[1] = flags = seeds = nullptr;
}

ms_status DevGraph::voronoi(ms_ctx* c, const std::vector<int>& sd, std::vector<int>& label,
                            std::vector<double>& dist) {
  if (hipSetDevice(c->dev.device) != hipSuccess) return MS_E_DEVICE;
  hipStream_t st = c->stream;
  const int ns = int(sd.size());
  const unsigned nb = unsigned((n + 255) / 256);
  if (hipMemcpyAsync(seeds, sd.data(), ns * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess)
    return MS_E_DEVICE;
  k_vor_init<<<nb, 256, 0, st>>>(n, seeds, ns, d[0], l[0]);
  if (ns) k_vor_seeds<<<unsigned((ns + 255) / 256), 256, 0, st>>>(seeds, ns, d[0], l[0]);
  int cur = 0;
  std::vector<int> hf(kSweepChunk);
  for (int sweeps = 0;; sweeps += kSweepChunk) {
    if (sweeps > 4 * n + 4 * kSweepChunk) return MS_E_DEVICE;  // cannot happen with positive costs
    if (hipMemsetAsync(flags, 0, kSweepChunk * sizeof(int), st) != hipSuccess) return MS_E_DEVICE;
    for (int q = 0; q < kSweepChunk; ++q) {
      k_vor_sweep<<<nb, 256, 0, st>>>(n, ptr, idx, len, d[cur], l[cur], d[1 - cur], l[1 - cur], flags + q);
      cur = 1 - cur;
    }
    if (hipMemcpyAsync(hf.data(), flags, kSweepChunk * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return MS_E_DEVICE;
    if (hf[kSweepChunk - 1] == 0) break;
  }
  label.resize(n);
  dist.resize(n);
  if (hipMemcpyAsync(label.data(), l[cur], n * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(dist.data(), d[cur], n * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess)
    return MS_E_DEVICE;
  return MS_OK;
}

}  // namespace ms
