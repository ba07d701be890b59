// Host construction of the sparse geometry- and material-aware basis
// (Sec. 3.4-3.6 of the paper).
//
//  1. Per-tet stiffness w_e = E_e; tets touching a vertex shared by tets of
//     different materials get the jump penalty w_e = jump * min(E) for the
//     distance computation (Sec. 3.6.2).
//  2. Stiffness-weighted geodesic distance on the vertex graph: each edge
//     costs its length times sqrt(w_ref / w_edge) (w_edge = mean w of the
//     tets around it), so distance grows slowly in stiff material and fast
//     across material jumps.  (The paper computes the distance with heat
//     diffusion and a stiffness-weighted Laplacian; the graph metric is the
//     same idea at a fraction of the cost -- see the design notes.)
//  3. K-means by Lloyd relaxation under that metric (the nearest-seed
//     searches by Dijkstra on the host, or by Jacobi sweeps on the GPU when
//     the build has a device: the same labels and distances), initialised by
//     kmeans++ with oversampling; every prune_every iterations the prune_n
//     smallest clusters with median volume > prune_ratio x own volume are
//     deleted (Sec. 3.6.3).  Tets take the label of the majority of their
//     vertices; a seed moves to the partition vertex nearest the
//     partition's volume centroid.
//  4. For each partition i: subdomain T_i = i and its face neighbours; solve
//     the stiffness-weighted biharmonic K u = 0, K = L M^-1 L assembled on
//     T_i, with u = 1 at i's centroid vertex, u = 0 at the neighbours'
//     centroid vertices, on the internal boundary of T_i and at Dirichlet
//     vertices (Sec. 3.5, 3.5.1); clip u_pos = max(u, 0).
//  5. With Dirichlet vertices, u_DBC: the same solve on the partitions that
//     hold Dirichlet vertices plus their neighbours with u = 1 at the
//     Dirichlet vertices and u = 0 at the other centroids.
//  6. Partition of unity phi_i = u_pos,i / (sum_j u_pos,j + u_DBC); handle
//     origins are the partition volume centroids.  A free vertex that no
//     clipped solution reaches gets weight 1 in its own partition, so the
//     partition of unity (hence linear precision) holds at every vertex.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <queue>
#include <random>
#include <thread>
#include <unordered_map>

#include "ms_internal.h"
#include "sparse_chol.h"

namespace ms {

namespace {

struct Graph {
  std::vector<int> ptr, idx;
  std::vector<double> len;
};

Graph build_graph(const ms_ctx* c, const std::vector<double>& w, double wref) {
  const int64_t n = c->n, T = c->T;
  std::vector<std::vector<std::pair<int, double>>> adj(n);  // neighbour, accumulated w
  std::vector<std::unordered_map<int, std::pair<double, int>>> acc(n);
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        if (a == b) continue;
        int i = c->h_tets[4 * t + a], j = c->h_tets[4 * t + b];
        auto& e = acc[i][j];
        e.first += w[t];
        e.second += 1;
      }
  Graph G;
  G.ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) G.ptr[i + 1] = G.ptr[i] + int(acc[i].size());
  G.idx.resize(G.ptr[n]);
  G.len.resize(G.ptr[n]);
  for (int64_t i = 0; i < n; ++i) {
    std::vector<std::pair<int, double>> row;
    for (auto& kv : acc[i]) row.push_back({kv.first, kv.second.first / kv.second.second});
    std::sort(row.begin(), row.end());
    int k = G.ptr[i];
    for (auto& pr : row) {
      const int j = pr.first;
      double L = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double dd = c->h_rest[3 * i + d] - c->h_rest[3 * j + d];
        L += dd * dd;
      }
      G.idx[k] = j;
      G.len[k] = std::sqrt(L) * std::sqrt(wref / std::max(pr.second, 1e-300));
      ++k;
    }
  }
  return G;
}

// Multi-source Dijkstra: label and distance of the nearest seed.
void voronoi(const Graph& G, const std::vector<int>& seeds, std::vector<int>& label, std::vector<double>& dist) {
  const int n = int(G.ptr.size()) - 1;
  label.assign(n, -1);
  dist.assign(n, INFINITY);
  using QE = std::pair<double, int>;
  std::priority_queue<QE, std::vector<QE>, std::greater<QE>> q;
  for (int s = 0; s < int(seeds.size()); ++s) {
    dist[seeds[s]] = 0.0;
    label[seeds[s]] = s;
    q.push({0.0, seeds[s]});
  }
  while (!q.empty()) {
    auto [d, v] = q.top();
    q.pop();
    if (d > dist[v]) continue;
    for (int k = G.ptr[v]; k < G.ptr[v + 1]; ++k) {
      const int w = G.idx[k];
      const double nd = d + G.len[k];
      if (nd < dist[w] || (nd == dist[w] && label[v] < label[w])) {
        dist[w] = nd;
        label[w] = label[v];
        q.push({nd, w});
      }
    }
  }
}

struct Partitioning {
  std::vector<int> tet_label;  // [T]
  int m = 0;
  ms_status err = MS_OK;
};

// nearest-seed labels and distances (host Dijkstra, or the device sweeps)
using VoronoiFn = std::function<ms_status(const std::vector<int>&, std::vector<int>&, std::vector<double>&)>;

Partitioning kmeans(const ms_ctx* c, const Graph& G, const ms_basis_params& P, const VoronoiFn& vor) {
  const int64_t n = c->n, T = c->T;
  std::mt19937_64 rng(P.seed);
  const int m_target = std::max(1, P.n_handles);
  std::vector<int> seeds;
  std::vector<int> label;
  std::vector<double> dist;
  if (P.lattice_seeding) {
    // seeds: vertices nearest to the points of a regular lattice with about
    // m_target points inside the bounding box (kept only if a vertex lies close)
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < n; ++v)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], c->h_rest[3 * v + d]);
        hi[d] = std::max(hi[d], c->h_rest[3 * v + d]);
      }
    const int k = std::max(1, int(std::round(std::cbrt(double(m_target)))));
    std::vector<char> used(n, 0);
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b)
        for (int e = 0; e < k; ++e) {
          const double p[3] = {lo[0] + (a + 0.5) * (hi[0] - lo[0]) / k, lo[1] + (b + 0.5) * (hi[1] - lo[1]) / k,
                               lo[2] + (e + 0.5) * (hi[2] - lo[2]) / k};
          int best = -1;
          double bd = 1e300;
          for (int64_t v = 0; v < n; ++v) {
            double dd = 0;
            for (int d = 0; d < 3; ++d) dd += (c->h_rest[3 * v + d] - p[d]) * (c->h_rest[3 * v + d] - p[d]);
            if (dd < bd) bd = dd, best = int(v);
          }
          if (best >= 0 && !used[best]) {
            used[best] = 1;
            seeds.push_back(best);
          }
        }
  } else {
    // kmeans++ with oversampling
    const int k0 = std::max(m_target, int(std::ceil(P.oversample * m_target)));
    seeds.push_back(int(rng() % uint64_t(n)));
    while (int(seeds.size()) < std::min<int64_t>(k0, n)) {
      if (ms_status e = vor(seeds, label, dist)) {
        Partitioning bad;
        bad.err = e;
        return bad;
      }
      double tot = 0.0;
      for (int64_t v = 0; v < n; ++v) tot += std::isfinite(dist[v]) ? dist[v] * dist[v] : 0.0;
      if (!(tot > 0)) break;
      double r = std::uniform_real_distribution<double>(0.0, tot)(rng);
      int pick = int(n - 1);
      for (int64_t v = 0; v < n; ++v) {
        r -= std::isfinite(dist[v]) ? dist[v] * dist[v] : 0.0;
        if (r <= 0) {
          pick = int(v);
          break;
        }
      }
      seeds.push_back(pick);
    }
  }
  std::vector<int> tl(T, 0);
  // Voronoi cells of the seeds, then every tet takes the majority label of
  // its vertices (ties: the nearer vertex)
  ms_status verr = MS_OK;
  auto label_tets = [&]() {
    if (ms_status e = vor(seeds, label, dist)) {
      verr = e;
      return;
    }
    for (int64_t t = 0; t < T; ++t) {
      int best = -1, bc = 0;
      double bd = 1e300;
      for (int a = 0; a < 4; ++a) {
        const int la = label[c->h_tets[4 * t + a]];
        int cnt = 0;
        double dmin = 1e300;
        for (int b = 0; b < 4; ++b)
          if (label[c->h_tets[4 * t + b]] == la) {
            ++cnt;
            dmin = std::min(dmin, dist[c->h_tets[4 * t + b]]);
          }
        if (cnt > bc || (cnt == bc && dmin < bd)) best = la, bc = cnt, bd = dmin;
      }
      tl[t] = best < 0 ? 0 : best;
    }
  };
  bool labels_stale = false;  // tl refers to a seed set that pruning has since changed
  for (int it = 0; it < std::max(1, P.max_lloyd); ++it) {
    label_tets();
    if (verr) break;
    labels_stale = false;
    const int k = int(seeds.size());
    std::vector<double> vol(k, 0.0), cen(3 * k, 0.0);
    for (int64_t t = 0; t < T; ++t) {
      const int l = tl[t];
      vol[l] += c->h_vol[t];
      for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) cen[3 * l + d] += c->h_vol[t] * 0.25 * c->h_rest[3 * c->h_tets[4 * t + a] + d];
    }
    // pruning
    bool pruned = false;
    if (!P.lattice_seeding && k > m_target && P.prune_every > 0 && (it + 1) % P.prune_every == 0) {
      std::vector<double> sv(vol);
      std::nth_element(sv.begin(), sv.begin() + k / 2, sv.end());
      const double med = sv[k / 2];
      std::vector<int> cand;
      for (int l = 0; l < k; ++l)
        if (med > P.prune_ratio * vol[l]) cand.push_back(l);
      std::sort(cand.begin(), cand.end(), [&](int a, int b) { return vol[a] < vol[b] || (vol[a] == vol[b] && a < b); });
      int del = std::min<int>(std::min(P.prune_n, int(cand.size())), k - m_target);
      if (del > 0) {
        std::vector<char> kill(k, 0);
        for (int q = 0; q < del; ++q) kill[cand[q]] = 1;
        std::vector<int> ns;
        for (int l = 0; l < k; ++l)
          if (!kill[l]) ns.push_back(seeds[l]);
        seeds.swap(ns);
        pruned = true;
      }
    }
    if (pruned) {
      labels_stale = true;
      continue;
    }
    // move each seed to the partition vertex nearest the volume centroid
    std::vector<int> nseeds(seeds);
    std::vector<double> bestd(k, 1e300);
    for (int64_t t = 0; t < T; ++t) {
      const int l = tl[t];
      if (!(vol[l] > 0)) continue;
      for (int a = 0; a < 4; ++a) {
        const int v = c->h_tets[4 * t + a];
        if (label[v] != l) continue;
        double dd = 0;
        for (int d = 0; d < 3; ++d) {
          const double q = c->h_rest[3 * v + d] - cen[3 * l + d] / vol[l];
          dd += q * q;
        }
        if (dd < bestd[l] || (dd == bestd[l] && v < nseeds[l])) bestd[l] = dd, nseeds[l] = v;
      }
    }
    if (nseeds == seeds && !(int(seeds.size()) > m_target && !P.lattice_seeding)) break;
    seeds.swap(nseeds);
  }
  // the Lloyd budget can end right after a pruning round: label the tets
  // of the remaining seeds before compacting
  if (labels_stale && !verr) label_tets();
  if (verr) {
    Partitioning bad;
    bad.err = verr;
    return bad;
  }
  // compact labels (drop empty partitions)
  std::vector<int> remap(seeds.size(), -1);
  Partitioning out;
  out.tet_label.resize(T);
  for (int64_t t = 0; t < T; ++t) {
    int& r = remap[tl[t]];
    if (r < 0) r = out.m++;
    out.tet_label[t] = r;
  }
  return out;
}

// Stiffness-weighted P1 Laplacian on a set of tets in local vertex numbering;
// also returns lumped vertex volumes.
void local_laplacian(const ms_ctx* c, const std::vector<int64_t>& tets, const std::vector<int>& loc, int nl,
                     const std::vector<double>& w, Csr& L, std::vector<double>& mv) {
  std::vector<std::map<int, double>> rows(nl);
  mv.assign(nl, 0.0);
  for (int64_t t : tets) {
    const double* Dm = &c->h_Dminv[9 * t];
    double beta[4][3];
    for (int j = 0; j < 3; ++j) {
      beta[1][j] = Dm[j];
      beta[2][j] = Dm[3 + j];
      beta[3][j] = Dm[6 + j];
      beta[0][j] = -(beta[1][j] + beta[2][j] + beta[3][j]);
    }
    const double V = c->h_vol[t], we = w[t];
    int li[4];
    for (int a = 0; a < 4; ++a) li[a] = loc[c->h_tets[4 * t + a]];
    for (int a = 0; a < 4; ++a) {
      mv[li[a]] += V / 4.0;
      for (int b = 0; b < 4; ++b) {
        const double g = beta[a][0] * beta[b][0] + beta[a][1] * beta[b][1] + beta[a][2] * beta[b][2];
        rows[li[a]][li[b]] += we * V * g;
      }
    }
  }
  L.n = nl;
  L.ptr.assign(nl + 1, 0);
  for (int i = 0; i < nl; ++i) L.ptr[i + 1] = L.ptr[i] + int(rows[i].size());
  L.idx.resize(L.ptr[nl]);
  L.val.resize(L.ptr[nl]);
  for (int i = 0; i < nl; ++i) {
    int k = L.ptr[i];
    for (auto& kv : rows[i]) {
      L.idx[k] = kv.first;
      L.val[k] = kv.second;
      ++k;
    }
  }
}

// K = L diag(1/mv) L restricted to the free rows/cols; rhs = -K_fc u_c.
void bilaplacian_system(const Csr& L, const std::vector<double>& mv, const std::vector<char>& fixed,
                        const std::vector<double>& uval, Csr& K, std::vector<double>& rhs, std::vector<int>& fidx) {
  const int nl = L.n;
  std::vector<int> fpos(nl, -1);
  fidx.clear();
  for (int i = 0; i < nl; ++i)
    if (!fixed[i]) {
      fpos[i] = int(fidx.size());
      fidx.push_back(i);
    }
  const int nf = int(fidx.size());
  K.n = nf;
  K.ptr.assign(nf + 1, 0);
  K.idx.clear();
  K.val.clear();
  rhs.assign(nf, 0.0);
  std::vector<double> acc(nl, 0.0);
  std::vector<int> touched;
  std::vector<char> mark(nl, 0);
  for (int r = 0; r < nf; ++r) {
    const int i = fidx[r];
    touched.clear();
    for (int a = L.ptr[i]; a < L.ptr[i + 1]; ++a) {
      const int k = L.idx[a];
      const double lik = L.val[a] / mv[k];
      for (int b = L.ptr[k]; b < L.ptr[k + 1]; ++b) {
        const int j = L.idx[b];
        if (!mark[j]) {
          mark[j] = 1;
          touched.push_back(j);
        }
        acc[j] += lik * L.val[b];
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int j : touched) {
      if (fpos[j] >= 0) {
        K.idx.push_back(fpos[j]);
        K.val.push_back(acc[j]);
      } else {
        rhs[r] -= acc[j] * uval[j];
      }
      acc[j] = 0.0;
      mark[j] = 0;
    }
    K.ptr[r + 1] = int(K.idx.size());
  }
}

struct LocalResult {
  std::vector<int64_t> verts;  // global vertex ids
  std::vector<double> u;       // clipped values
  ms_status err = MS_OK;       // device failure of a GPU solve
  bool gpu = false;            // solved on the GPU
};

std::mutex g_gpu_solve;  // one dense GPU solve at a time (worker threads share the context's stream)

// Solves the constrained biharmonic on a set of tets: u = val on `ones`
// (value 1) and zero on `zeros` plus the internal boundary.
using FaceMap = std::map<std::array<int, 3>, int>;

FaceMap mesh_faces(const ms_ctx* c) {
  FaceMap fc;
  for (int64_t t = 0; t < c->T; ++t) {
    const int32_t* v = &c->h_tets[4 * t];
    const int f[4][3] = {{v[1], v[2], v[3]}, {v[0], v[2], v[3]}, {v[0], v[1], v[3]}, {v[0], v[1], v[2]}};
    for (auto& ff : f) {
      std::array<int, 3> key = {ff[0], ff[1], ff[2]};
      std::sort(key.begin(), key.end());
      fc[key]++;
    }
  }
  return fc;
}

LocalResult local_biharmonic(const ms_ctx* c, const std::vector<int64_t>& tets, const std::vector<int>& ones,
                             const std::vector<int>& zeros, const std::vector<char>& is_dbc,
                             const std::vector<double>& w, const FaceMap& mfaces) {
  LocalResult R;
  std::vector<int> loc(c->n, -1);
  for (int64_t t : tets)
    for (int a = 0; a < 4; ++a) {
      const int v = c->h_tets[4 * t + a];
      if (loc[v] < 0) {
        loc[v] = int(R.verts.size());
        R.verts.push_back(v);
      }
    }
  const int nl = int(R.verts.size());
  Csr L;
  std::vector<double> mv;
  local_laplacian(c, tets, loc, nl, w, L, mv);
  std::vector<char> fixed(nl, 0);
  std::vector<double> uval(nl, 0.0);
  // internal boundary: faces of the subdomain not shared inside it but shared in the mesh
  {
    std::map<std::array<int, 3>, int> fc;
    for (int64_t t : tets) {
      const int32_t* v = &c->h_tets[4 * t];
      const int f[4][3] = {{v[1], v[2], v[3]}, {v[0], v[2], v[3]}, {v[0], v[1], v[3]}, {v[0], v[1], v[2]}};
      for (auto& ff : f) {
        std::array<int, 3> key = {ff[0], ff[1], ff[2]};
        std::sort(key.begin(), key.end());
        fc[key]++;
      }
    }
    for (auto& kv : fc) {
      if (kv.second != 1) continue;
      // boundary face of the subdomain: internal if the mesh has another tet on it
      auto it = mfaces.find(kv.first);
      if (it != mfaces.end() && it->second == 2)
        for (int q = 0; q < 3; ++q) fixed[loc[kv.first[q]]] = 1;
    }
  }
  for (int i = 0; i < nl; ++i)
    if (is_dbc[R.verts[i]]) fixed[i] = 1;
  for (int v : zeros)
    if (loc[v] >= 0) fixed[loc[v]] = 1, uval[loc[v]] = 0.0;
  for (int v : ones)
    if (loc[v] >= 0) fixed[loc[v]] = 1, uval[loc[v]] = 1.0;
  Csr K;
  std::vector<double> rhs;
  std::vector<int> fidx;
  bilaplacian_system(L, mv, fixed, uval, K, rhs, fidx);
  std::vector<double> u(uval);
  if (K.n > 0) {
    bool done = false;
    if (c->basis_gpu_min > 0 && K.n >= c->basis_gpu_min) {
      // large subdomain: dense Cholesky on the GPU (falls back to the host
      // factorisation if a pivot is not positive)
      std::vector<double> x(rhs);
      bool ok = false;
      std::lock_guard<std::mutex> lk(g_gpu_solve);
      R.err = dense_spd_solve(const_cast<ms_ctx*>(c), K.n, K.ptr.data(), K.idx.data(), K.val.data(), x.data(), &ok);
      if (!R.err && ok) {
        rhs.swap(x);
        done = R.gpu = true;
      }
    }
    if (!done && !R.err) {
      EnvelopeCholesky ch;
      ch.factor(K);
      ch.solve(rhs);
    }
    for (int r = 0; r < K.n; ++r) u[fidx[r]] = rhs[r];
  }
  R.u.resize(nl);
  for (int i = 0; i < nl; ++i) R.u[i] = std::max(0.0, std::isfinite(u[i]) ? u[i] : 0.0);
  return R;
}

}  // namespace

ms_status build_basis_host(ms_ctx* c, const ms_basis_params& P, Basis& B) {
  const int64_t n = c->n, T = c->T;
  if (c->h_E.empty()) return fail(c, MS_E_ORDER, "material not uploaded");
  // 1. stiffness with jump penalty
  double emin = 1e300;
  for (double e : c->h_E) emin = std::min(emin, e);
  std::vector<double> vmin(n, 1e300), vmax(n, 0.0);
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a) {
      const int v = c->h_tets[4 * t + a];
      vmin[v] = std::min(vmin[v], c->h_E[t]);
      vmax[v] = std::max(vmax[v], c->h_E[t]);
    }
  std::vector<double> wdist(c->h_E);
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a) {
      const int v = c->h_tets[4 * t + a];
      if (vmax[v] > vmin[v] * (1.0 + 1e-12)) wdist[t] = P.jump_penalty * emin;
    }
  std::vector<double> sw(wdist);
  std::nth_element(sw.begin(), sw.begin() + T / 2, sw.end());
  const double wref = sw[T / 2];
  // 2-3. geodesic K-means partitioning
  const auto t_part = std::chrono::steady_clock::now();
  Graph G = build_graph(c, wdist, wref);
  // with a device, the nearest-seed searches run on it (same result)
  DevGraph dg;
  const bool dev_vor = c->basis_gpu_min > 0;
  if (dev_vor) {
    if (ms_status e = dg.upload(c, G.ptr, G.idx, G.len)) {
      dg.release(c);
      return fail(c, e, "basis graph upload failed");
    }
  }
  auto vor = [&](const std::vector<int>& sd, std::vector<int>& lab, std::vector<double>& dst) -> ms_status {
    if (dev_vor) return dg.voronoi(c, sd, lab, dst);
    voronoi(G, sd, lab, dst);
    return MS_OK;
  };
  Partitioning part = kmeans(c, G, P, vor);
  if (dev_vor) dg.release(c);
  if (part.err) return fail(c, part.err, "geodesic Voronoi on the GPU failed");
  const double part_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_part).count();
  const int m = part.m;
  // partition geometry: volume centroid and centroid vertex
  std::vector<double> pvol(m, 0.0), pcen(3 * m, 0.0);
  std::vector<std::vector<int64_t>> ptets(m);
  for (int64_t t = 0; t < T; ++t) {
    const int l = part.tet_label[t];
    ptets[l].push_back(t);
    pvol[l] += c->h_vol[t];
    for (int a = 0; a < 4; ++a)
      for (int d = 0; d < 3; ++d) pcen[3 * l + d] += c->h_vol[t] * 0.25 * c->h_rest[3 * c->h_tets[4 * t + a] + d];
  }
  for (int l = 0; l < m; ++l)
    for (int d = 0; d < 3; ++d) pcen[3 * l + d] /= pvol[l];
  std::vector<char> is_dbc(n, 0);
  for (int v : c->h_dbc) is_dbc[v] = 1;
  // vertex -> set of partitions of its tets
  std::vector<std::vector<int>> vparts(n);
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a) {
      auto& vp = vparts[c->h_tets[4 * t + a]];
      const int l = part.tet_label[t];
      if (std::find(vp.begin(), vp.end(), l) == vp.end()) vp.push_back(l);
    }
  std::vector<int> cvert(m, -1);
  {
    std::vector<double> best(m, 1e300), best_any(m, 1e300);
    std::vector<int> any(m, -1);
    for (int64_t v = 0; v < n; ++v) {
      if (is_dbc[v]) continue;
      for (int l : vparts[v]) {
        double dd = 0;
        for (int d = 0; d < 3; ++d) dd += (c->h_rest[3 * v + d] - pcen[3 * l + d]) * (c->h_rest[3 * v + d] - pcen[3 * l + d]);
        if (vparts[v].size() == 1 && dd < best[l]) best[l] = dd, cvert[l] = int(v);
        if (dd < best_any[l]) best_any[l] = dd, any[l] = int(v);
      }
    }
    for (int l = 0; l < m; ++l)
      if (cvert[l] < 0) cvert[l] = any[l];
  }
  // 4. face adjacency of partitions
  std::vector<std::vector<int>> nbr(m);
  {
    std::map<std::array<int, 3>, std::vector<int>> fp;
    for (int64_t t = 0; t < T; ++t) {
      const int32_t* v = &c->h_tets[4 * t];
      const int f[4][3] = {{v[1], v[2], v[3]}, {v[0], v[2], v[3]}, {v[0], v[1], v[3]}, {v[0], v[1], v[2]}};
      for (auto& ff : f) {
        std::array<int, 3> key = {ff[0], ff[1], ff[2]};
        std::sort(key.begin(), key.end());
        fp[key].push_back(part.tet_label[t]);
      }
    }
    for (auto& kv : fp)
      if (kv.second.size() == 2 && kv.second[0] != kv.second[1]) {
        const int a = kv.second[0], b = kv.second[1];
        if (std::find(nbr[a].begin(), nbr[a].end(), b) == nbr[a].end()) nbr[a].push_back(b);
        if (std::find(nbr[b].begin(), nbr[b].end(), a) == nbr[b].end()) nbr[b].push_back(a);
      }
    for (auto& v : nbr) std::sort(v.begin(), v.end());
  }
  // 4-5. local solves (one task per partition, plus the Dirichlet basis)
  const bool has_dbc = !c->h_dbc.empty();
  const int ntask = m + (has_dbc ? 1 : 0);
  std::vector<LocalResult> res(ntask);
  const FaceMap mfaces = mesh_faces(c);
  auto task = [&](int i) {
    std::vector<int64_t> tets;
    std::vector<int> ones, zeros;
    std::vector<char> in(m, 0);
    if (i < m) {
      in[i] = 1;
      for (int j : nbr[i]) in[j] = 1;
      ones.push_back(cvert[i]);
      for (int j : nbr[i]) zeros.push_back(cvert[j]);
    } else {
      for (int v : c->h_dbc)
        for (int l : vparts[v]) in[l] = 1;
      std::vector<char> core(in);
      for (int l = 0; l < m; ++l)
        if (core[l])
          for (int j : nbr[l]) in[j] = 1;
      for (int l = 0; l < m; ++l)
        if (in[l] && !core[l]) zeros.push_back(cvert[l]);
    }
    for (int l = 0; l < m; ++l)
      if (in[l]) tets.insert(tets.end(), ptets[l].begin(), ptets[l].end());
    std::sort(tets.begin(), tets.end());
    if (i < m) {
      res[i] = local_biharmonic(c, tets, ones, zeros, is_dbc, c->h_E, mfaces);
    } else {
      // Dirichlet basis: u = 1 on Dirichlet vertices (fixed as "ones")
      std::vector<char> no_dbc(n, 0);
      std::vector<int> dv(c->h_dbc.begin(), c->h_dbc.end());
      res[i] = local_biharmonic(c, tets, dv, zeros, no_dbc, c->h_E, mfaces);
    }
  };
  int nth = P.n_threads > 0 ? P.n_threads : int(std::max(1u, std::thread::hardware_concurrency()));
  nth = std::min(nth, ntask);
  std::atomic<int> next(0);
  // largest subdomains first for load balance
  std::vector<int> order(ntask);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> cost(ntask, 0.0);
  for (int i = 0; i < m; ++i) {
    cost[i] = double(ptets[i].size());
    for (int j : nbr[i]) cost[i] += double(ptets[j].size());
  }
  if (has_dbc) cost[m] = 1e300;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<std::thread> pool;
  for (int k = 0; k < nth; ++k)
    pool.emplace_back([&]() {
      for (int q = next++; q < ntask; q = next++) task(order[q]);
    });
  for (auto& th : pool) th.join();
  if (std::getenv("MS_VERBOSE"))
    std::fprintf(stderr, "[ms] basis: partitioning %.3f s, local solves %.3f s (%d tasks)\n", part_s,
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t_part).count() - part_s, ntask);
  c->basis_gpu_solves = 0;
  for (auto& rr : res) {
    if (rr.err) return fail(c, rr.err, "local basis solve on the GPU failed");
    c->basis_gpu_solves += rr.gpu ? 1 : 0;
  }
  // 6. partition of unity
  std::vector<double> denom(n, 0.0);
  for (int i = 0; i < ntask; ++i)
    for (size_t k = 0; k < res[i].verts.size(); ++k) denom[res[i].verts[k]] += res[i].u[k];
  std::vector<std::vector<std::pair<int, double>>> rows(n);
  for (int i = 0; i < m; ++i)
    for (size_t k = 0; k < res[i].verts.size(); ++k) {
      const int64_t v = res[i].verts[k];
      const double u = res[i].u[k];
      if (u > 0.0 && denom[v] > 0.0) rows[v].push_back({i, u / denom[v]});
    }
  // Vertices that no clipped solution reaches (possible near the mesh
  // boundary, where the natural boundary condition lets u dip below zero)
  // and that are not Dirichlet-bound are given weight 1 in the lowest-indexed
  // partition of their tets, which keeps the partition of unity everywhere.
  for (int64_t v = 0; v < n; ++v)
    if (!(denom[v] > 0.0) && !is_dbc[v] && !vparts[v].empty())
      rows[v].push_back({*std::min_element(vparts[v].begin(), vparts[v].end()), 1.0});
  // Optional stiff limit: constant weights on each connected set of stiff
  // tets (the average over its free vertices, in vertex order), so that
  // every handle moves a stiff inclusion affinely instead of bending it.
  if (P.rigid_contrast > 0.0) {
    std::vector<int64_t> root(n);
    std::iota(root.begin(), root.end(), int64_t(0));
    auto find = [&](int64_t a) {
      while (root[a] != a) a = root[a] = root[root[a]];
      return a;
    };
    std::vector<char> in_stiff(n, 0);
    for (int64_t t = 0; t < T; ++t) {
      if (!(c->h_E[t] >= P.rigid_contrast * emin)) continue;
      const int32_t* tv = &c->h_tets[4 * t];
      for (int a = 0; a < 4; ++a) in_stiff[tv[a]] = 1;
      for (int a = 1; a < 4; ++a) {
        const int64_t x = find(tv[0]), y = find(tv[a]);
        if (x != y) root[std::max(x, y)] = std::min(x, y);
      }
    }
    std::map<int64_t, std::vector<int64_t>> groups;  // root -> free vertices, ascending
    for (int64_t v = 0; v < n; ++v)
      if (in_stiff[v] && !is_dbc[v]) groups[find(v)].push_back(v);
    for (auto& kv : groups) {
      std::map<int, double> sum;
      for (int64_t v : kv.second)
        for (auto& pr : rows[v]) sum[pr.first] += pr.second;
      std::vector<std::pair<int, double>> avg;
      for (auto& hw : sum) avg.push_back({hw.first, hw.second / double(kv.second.size())});
      for (int64_t v : kv.second) rows[v] = avg;
    }
  }
  B.m = m;
  B.origins = pcen;
  B.vptr.assign(n + 1, 0);
  for (int64_t v = 0; v < n; ++v) {
    std::sort(rows[v].begin(), rows[v].end());
    B.vptr[v + 1] = B.vptr[v] + int64_t(rows[v].size());
  }
  B.nnz = B.vptr[n];
  B.vhandle.resize(B.nnz);
  B.vphi.resize(B.nnz);
  for (int64_t v = 0; v < n; ++v) {
    int64_t k = B.vptr[v];
    for (auto& pr : rows[v]) {
      B.vhandle[k] = pr.first;
      B.vphi[k] = pr.second;
      ++k;
    }
  }
  B.part = part.tet_label;
  return MS_OK;
}

}  // namespace ms

// ---------------------------------------------------------------------------
// Host-only entry points (no device needed).
// ---------------------------------------------------------------------------
struct ms_basis {
  ms::Basis B;
};

extern "C" ms_status ms_basis_compute(int64_t n, const double* rest, int64_t T, const int32_t* tets, const double* E,
                                      int64_t n_dbc, const int32_t* dbc, const ms_basis_params* p, ms_basis** out) {
  if (!rest || !tets || !E || !out || n < 4 || T < 1 || (n_dbc > 0 && !dbc)) return MS_E_ARG;
  ms_ctx c;
  c.n = n;
  c.T = T;
  c.h_rest.assign(rest, rest + 3 * n);
  c.h_tets.assign(tets, tets + 4 * T);
  for (int64_t i = 0; i < 4 * T; ++i)
    if (tets[i] < 0 || tets[i] >= n) return MS_E_ARG;
  ms_status s = ms::mesh_geometry(&c);
  if (s) return s;
  c.h_E.assign(E, E + T);
  for (int64_t t = 0; t < T; ++t)
    if (!(E[t] > 0) || !std::isfinite(E[t])) return MS_E_ARG;
  for (int64_t i = 0; i < n_dbc; ++i)
    if (dbc[i] < 0 || dbc[i] >= n) return MS_E_ARG;
  c.h_dbc.assign(dbc, dbc + n_dbc);
  ms_basis_params P;
  if (p)
    P = *p;
  else
    ms_basis_defaults(&P);
  if (P.n_handles < 1 || P.n_handles > n) return MS_E_ARG;
  ms_basis* b = new ms_basis();
  s = ms::build_basis_host(&c, P, b->B);
  if (s) {
    delete b;
    return s;
  }
  *out = b;
  return MS_OK;
}

extern "C" ms_status ms_basis_get(const ms_basis* b, int32_t* m, int64_t* nnz, double* origins, int64_t* vptr,
                                  int32_t* vhandle, double* vphi, int32_t* part) {
  if (!b || !m || !nnz) return MS_E_ARG;
  const ms::Basis& B = b->B;
  *m = B.m;
  *nnz = int64_t(B.vhandle.size());
  if (origins) std::copy(B.origins.begin(), B.origins.end(), origins);
  if (vptr) std::copy(B.vptr.begin(), B.vptr.end(), vptr);
  if (vhandle) std::copy(B.vhandle.begin(), B.vhandle.end(), vhandle);
  if (vphi) std::copy(B.vphi.begin(), B.vphi.end(), vphi);
  if (part) std::copy(B.part.begin(), B.part.end(), part);
  return MS_OK;
}

extern "C" void ms_basis_free(ms_basis* b) { delete b; }
