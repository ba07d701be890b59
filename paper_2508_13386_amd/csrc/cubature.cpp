// Modal moment-fitting cubature for the elastic part of the subspace Hessian
// (Sec. 3.8, Subspace Hessian Integration; Alg. 3), host side.
//
//  * Basis functions are evaluated per tet as the mean of their vertex
//    weights phi_i over the tet's four vertices.
//  * For each partition p of the basis construction, the functions that
//    touch p (sorted handle ids) give the degree-2 moment conditions: rows
//    1, u_i and u_i u_j (i <= j, lexicographic).  Column e of A holds the
//    values at tet e; the target is b = A V (volume-weighted sum over all of
//    the partition's tets).
//  * Alg. 3: n_init tets drawn uniformly, non-negative least squares on the
//    drawn columns, and while ||A w - b|| / ||b|| > tol, n_add more tets drawn
//    without replacement with probability proportional to (A_k^T r)^2.
//  * NNLS is Lawson and Hanson's active-set method (Solving Least Squares
//    Problems, 1974, ch. 23) with the least-squares subproblem kept as an
//    incrementally updated QR (a Householder reflector when a column enters,
//    Givens rotations restoring the triangle when one leaves).
//    The solver continues from its current passive set when a round adds
//    candidates.
//  * Draws come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as
//    a counter-based generator: draw j of partition p takes the state
//    seed + (2^32 p + j + 1) * 0x9E3779B97F4A7C15 through the reference
//    finaliser; the top 53 bits give a uniform double in [0, 1).
//
// The device side (coarse.hip) integrates the elastic Hessian over the
// selected tets only: K = U^T (M + h^2 (B'' + D'')) U
//                       + h^2 sum_q (w_q / V_q) U_q^T H_q U_q.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "ms_internal.h"

namespace ms {
namespace {

uint64_t splitmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t seed, uint64_t counter) {
  const uint64_t z = splitmix64(seed + (counter + 1) * 0x9E3779B97F4A7C15ull);
  return double(z >> 11) * (1.0 / 9007199254740992.0);
}

// Draws `count` columns without replacement, probability proportional to
// rho over the columns not chosen yet, in column order.
void draw(std::vector<double> rho, std::vector<char>& chosen, int count, uint64_t seed, uint64_t pid,
          uint64_t& counter) {
  const size_t n = rho.size();
  for (size_t k = 0; k < n; ++k)
    if (chosen[k]) rho[k] = 0.0;
  std::vector<double> cum(n);
  for (int d = 0; d < count; ++d) {
    double tot = 0.0;
    for (size_t k = 0; k < n; ++k) cum[k] = (tot += rho[k]);
    if (!(tot > 0.0)) break;
    const double u = uniform01(seed, (pid << 32) + counter) * tot;
    ++counter;
    size_t k = size_t(std::upper_bound(cum.begin(), cum.end(), u) - cum.begin());
    k = std::min(k, n - 1);
    while (rho[k] == 0.0) --k;
    chosen[k] = 1;
    rho[k] = 0.0;
  }
}

// Lawson-Hanson NNLS on the columns of A (m x n, column-major) that are
// marked available; x (size n) is the current feasible point (zero outside
// the passive set) and is updated in place.  Every column is kept in the
// basis of the Householder QR of the passive columns (Q^T A, Q^T b), so the
// gradient of a candidate is the product of the tails of Q^T a_j and Q^T b:
// the residual is never formed by cancellation, which keeps the gradients
// meaningful down to relative residuals near round-off (the moment matrices
// are very ill-conditioned: the partition of unity makes their rows nearly
// dependent).
class Nnls {
 public:
  Nnls(int m, const double* A, const double* b, int n)
      : m_(m), n_(n), A_(A), b_(b), x_(n, 0.0), passive_(n, 0), cnorm_(n), QA_(size_t(m) * n), ready_(n, 0) {
    for (int j = 0; j < n_; ++j) cnorm_[j] = norm(A_ + size_t(j) * m_, m_);
    reset();
  }

  // Solves over the available columns, starting from the current state (x
  // is the least-squares solution on the passive columns).
  void solve(const std::vector<char>& avail) {
    std::vector<char> blocked(n_, 0);
    std::vector<double> z;
    // Each completed iteration lowers the residual in exact arithmetic; the
    // solve ends when one no longer does (round-off level, which also stops
    // the cycling that round-off can cause) or after maxit iterations.
    double rn = tail_norm();
    const int maxit = 10 * m_ + 100;
    for (int it = 0; it < maxit; ++it) {
      const int p = int(cols_.size());
      int t = -1;
      double best = 0.0;
      for (int j = 0; j < n_; ++j) {
        if (!avail[j] || passive_[j] || blocked[j]) continue;
        ready(j);
        const double* a = QA_.data() + size_t(j) * m_;
        double g = 0.0;
        for (int i = p; i < m_; ++i) g += a[i] * qtb_[i];
        if (g > best) best = g, t = j;
      }
      if (t < 0) return;
      if (!add(t)) {  // numerically dependent on the passive columns
        blocked[t] = 1;
        continue;
      }
      passive_[t] = 1;
      bool first = true;
      for (;;) {
        lsq(z);
        bool pos = true;
        for (size_t q = 0; q < cols_.size(); ++q) {
          if (!std::isfinite(z[q])) z[q] = 0.0;  // treated as leaving the passive set
          pos = pos && z[q] > 0.0;
        }
        if (pos) {
          for (size_t q = 0; q < cols_.size(); ++q) x_[cols_[q]] = z[q];
          std::fill(blocked.begin(), blocked.end(), 0);
          const double rn2 = tail_norm();
          if (!(rn2 < rn)) return;
          rn = rn2;
          break;
        }
        if (first && z[cols_.size() - 1] <= 0.0) {
          // the entering column cannot take a positive value (round-off):
          // drop it and keep x
          passive_[t] = 0;
          blocked[t] = 1;
          remove(int(cols_.size()) - 1);
          break;
        }
        first = false;
        double alpha = 1.0;
        for (size_t q = 0; q < cols_.size(); ++q)
          if (z[q] <= 0.0) {
            const double xj = x_[cols_[q]];
            alpha = std::min(alpha, xj - z[q] > 0.0 ? xj / (xj - z[q]) : 0.0);
          }
        std::vector<int> leave;  // positions, ascending
        for (size_t q = 0; q < cols_.size(); ++q) {
          const int j = cols_[q];
          const double xo = x_[j];
          // the column(s) that set alpha reach zero (up to round-off)
          const bool hit = z[q] <= 0.0 && (xo - z[q] > 0.0 ? xo / (xo - z[q]) : 0.0) <= alpha * (1.0 + 1e-12);
          x_[j] = xo + alpha * (z[q] - xo);
          if (hit || x_[j] <= 0.0) {
            x_[j] = 0.0;
            passive_[j] = 0;
            leave.push_back(int(q));
          }
        }
        for (size_t q = leave.size(); q-- > 0;) remove(leave[q]);
        std::fill(blocked.begin(), blocked.end(), 0);
        if (cols_.empty()) break;
      }
    }
  }

  const std::vector<double>& x() const { return x_; }

  double rel_residual() const {
    std::vector<double> r(b_, b_ + m_);
    for (int j = 0; j < n_; ++j)
      if (x_[j] != 0.0) {
        const double* a = A_ + size_t(j) * m_;
        for (int i = 0; i < m_; ++i) r[i] -= x_[j] * a[i];
      }
    const double bn = norm(b_, m_);
    return bn > 0.0 ? norm(r.data(), m_) / bn : 0.0;
  }

 private:
  static double dot(const double* a, const double* b, int m) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += a[i] * b[i];
    return s;
  }
  static double norm(const double* a, int m) { return std::sqrt(dot(a, a, m)); }

  // ||A x - b|| at the least-squares solution on the passive columns.
  double tail_norm() const {
    double s = 0.0;
    for (int i = int(cols_.size()); i < m_; ++i) s += qtb_[i] * qtb_[i];
    return std::sqrt(s);
  }

  void reset() {
    std::fill(ready_.begin(), ready_.end(), 0);
    touched_.clear();
    qtb_.assign(b_, b_ + m_);
    cols_.clear();
    R_.clear();
    ops_.clear();
  }

  // Brings column j of Q^T A up to date by replaying the transformations
  // applied so far (only columns that have been candidates are kept).
  void ready(int j) {
    if (ready_[j]) return;
    double* a = QA_.data() + size_t(j) * m_;
    std::copy(A_ + size_t(j) * m_, A_ + size_t(j + 1) * m_, a);
    for (const Op& o : ops_) apply(o, a);
    ready_[j] = 1;
    touched_.push_back(j);
  }

  // Removes the passive column at position q: the columns after it shift
  // left and Givens rotations of rows (k, k+1) restore R's triangle; every
  // current column and Q^T b take the same rotations.
  void remove(int q) {
    cols_.erase(cols_.begin() + q);
    R_.erase(R_.begin() + q);
    for (int k = q; k < int(cols_.size()); ++k) {
      const double a = R_[k][k], b = R_[k][k + 1];
      const double r = std::hypot(a, b);
      Op o;
      o.q = k;
      o.c = r > 0.0 ? a / r : 1.0;
      o.s = r > 0.0 ? b / r : 0.0;
      R_[k][k] = r;
      R_[k].pop_back();
      for (int kk = k + 1; kk < int(cols_.size()); ++kk) rotate(o, R_[kk].data());
      for (int jj : touched_) rotate(o, QA_.data() + size_t(jj) * m_);
      rotate(o, qtb_.data());
      ops_.push_back(std::move(o));
    }
  }

  // Appends column j to the QR of the passive columns and applies the new
  // reflector to every column and to Q^T b; false when the column's part
  // outside the passive span is negligible.
  bool add(int j) {
    const int p = int(cols_.size());
    if (p >= m_) return false;
    ready(j);
    const double* a = QA_.data() + size_t(j) * m_;
    double s = 0.0;
    for (int i = p; i < m_; ++i) s += a[i] * a[i];
    s = std::sqrt(s);
    if (!(s > 1e-14 * cnorm_[j])) return false;
    const double alpha = a[p] > 0.0 ? -s : s;
    std::vector<double> v(m_, 0.0);
    v[p] = a[p] - alpha;
    for (int i = p + 1; i < m_; ++i) v[i] = a[i];
    const double vn = norm(v.data(), m_);
    for (int i = p; i < m_; ++i) v[i] /= vn;
    std::vector<double> rcol(a, a + p);
    rcol.push_back(alpha);
    R_.push_back(std::move(rcol));
    Op o;
    o.q = p;
    o.v = std::move(v);
    for (int k : touched_) apply(o, QA_.data() + size_t(k) * m_);
    apply(o, qtb_.data());
    ops_.push_back(std::move(o));
    cols_.push_back(j);
    return true;
  }

  // An orthogonal transformation of Q^T: a Householder reflector I - 2 v v^T
  // (v nonzero from row q on) or a rotation [c s; -s c] of rows (q, q+1).
  struct Op {
    int q = 0;
    std::vector<double> v;  // empty for a rotation
    double c = 1.0, s = 0.0;
  };

  void apply(const Op& o, double* a) const {
    if (o.v.empty()) {
      rotate(o, a);
      return;
    }
    double s = 0.0;
    for (int i = o.q; i < m_; ++i) s += o.v[i] * a[i];
    s *= 2.0;
    for (int i = o.q; i < m_; ++i) a[i] -= s * o.v[i];
  }

  static void rotate(const Op& o, double* a) {
    const double y0 = a[o.q], y1 = a[o.q + 1];
    a[o.q] = o.c * y0 + o.s * y1;
    a[o.q + 1] = -o.s * y0 + o.c * y1;
  }

  // z = argmin || A_P z - b || by back substitution on R z = Q^T b.
  void lsq(std::vector<double>& z) const {
    const int p = int(cols_.size());
    z.assign(p, 0.0);
    for (int q = p - 1; q >= 0; --q) {
      double s = qtb_[q];
      for (int k = q + 1; k < p; ++k) s -= R_[k][q] * z[k];
      z[q] = s / R_[q][q];
    }
  }

  int m_, n_;
  const double* A_;
  const double* b_;
  std::vector<double> x_;
  std::vector<char> passive_;
  std::vector<double> cnorm_;             // column norms of A
  std::vector<double> QA_;                // Q^T A, column-major (columns in touched_)
  std::vector<char> ready_;               // column of QA_ is current
  std::vector<int> touched_;              // the current columns
  std::vector<Op> ops_;                   // transformations applied to Q^T, in order
  std::vector<double> qtb_;               // Q^T b
  std::vector<int> cols_;                 // passive columns in factorisation order
  std::vector<std::vector<double>> R_;    // R by columns
};

struct PartFit {
  std::vector<int32_t> tets;
  std::vector<double> w;
  double rel = 0.0;
};

// Alg. 3 on the tets `ids` of partition pid.
PartFit fit_partition(const std::vector<int32_t>& ids, const std::vector<double>& vol,
                      const std::vector<std::vector<std::pair<int, double>>>& ev, int64_t pid,
                      const CubatureParams& P) {
  const int ne = int(ids.size());
  // functions touching the partition
  std::vector<int> hs;
  for (int e = 0; e < ne; ++e)
    for (auto& pr : ev[ids[e]])
      if (pr.second != 0.0) hs.push_back(pr.first);
  std::sort(hs.begin(), hs.end());
  hs.erase(std::unique(hs.begin(), hs.end()), hs.end());
  const int k = int(hs.size());
  const int m = 1 + k + k * (k + 1) / 2;
  std::vector<double> A(size_t(m) * ne, 0.0), b(m, 0.0), u(k);
  for (int e = 0; e < ne; ++e) {
    std::fill(u.begin(), u.end(), 0.0);
    for (auto& pr : ev[ids[e]]) {
      const int a = int(std::lower_bound(hs.begin(), hs.end(), pr.first) - hs.begin());
      if (a < k && hs[a] == pr.first) u[a] = pr.second;
    }
    double* col = A.data() + size_t(e) * m;
    int row = 0;
    col[row++] = 1.0;
    for (int a = 0; a < k; ++a) col[row++] = u[a];
    for (int a = 0; a < k; ++a)
      for (int c = a; c < k; ++c) col[row++] = u[a] * u[c];
  }
  for (int e = 0; e < ne; ++e) {
    const double* col = A.data() + size_t(e) * m;
    const double v = vol[ids[e]];
    for (int i = 0; i < m; ++i) b[i] += col[i] * v;
  }
  // weights in units of the mean tet volume
  const double scale = b[0] > 0.0 ? b[0] / ne : 1.0;
  std::vector<double> bs(m);
  for (int i = 0; i < m; ++i) bs[i] = b[i] / scale;
  std::vector<char> chosen(ne, 0);
  uint64_t counter = 0;
  draw(std::vector<double>(ne, 1.0), chosen, std::min(P.n_init, ne), P.seed, uint64_t(pid), counter);
  Nnls solver(m, A.data(), bs.data(), ne);
  double rel = 0.0;
  for (int round = 0; round <= P.max_rounds; ++round) {
    solver.solve(chosen);
    rel = solver.rel_residual();
    const bool all = std::all_of(chosen.begin(), chosen.end(), [](char c) { return c != 0; });
    if (rel <= P.tol || all || round == P.max_rounds) break;
    // rho_k = (A_k^T r)^2 with r = A w - b
    std::vector<double> r(m);
    for (int i = 0; i < m; ++i) r[i] = -bs[i];
    const std::vector<double>& x = solver.x();
    for (int e = 0; e < ne; ++e)
      if (x[e] != 0.0)
        for (int i = 0; i < m; ++i) r[i] += x[e] * A[size_t(e) * m + i];
    std::vector<double> rho(ne);
    for (int e = 0; e < ne; ++e) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += A[size_t(e) * m + i] * r[i];
      rho[e] = s * s;
    }
    draw(rho, chosen, P.n_add, P.seed, uint64_t(pid), counter);
  }
  PartFit out;
  out.rel = rel;
  const std::vector<double>& x = solver.x();
  for (int e = 0; e < ne; ++e)
    if (x[e] > 0.0) {
      out.tets.push_back(ids[e]);
      out.w.push_back(x[e] * scale);
    }
  return out;
}

}  // namespace

ms_status fit_cubature_host(int64_t n, const double* rest, int64_t T, const int32_t* tets, const int32_t* part,
                            const int64_t* vptr, const int32_t* vhandle, const double* vphi,
                            const CubatureParams& P, std::vector<int32_t>& sel, std::vector<double>& wts,
                            double* max_rel) {
  // tet volumes and per-tet basis values (handle, mean of phi over the 4 vertices)
  std::vector<double> vol(T);
  std::vector<std::vector<std::pair<int, double>>> ev(T);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t* tv = tets + 4 * t;
    const double* x0 = rest + 3 * int64_t(tv[0]);
    double d[3][3];
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < 3; ++i) d[a][i] = rest[3 * int64_t(tv[a + 1]) + i] - x0[i];
    const double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                       d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                       d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
    vol[t] = std::fabs(det) / 6.0;
    auto& row = ev[t];
    for (int a = 0; a < 4; ++a)
      for (int64_t k = vptr[tv[a]]; k < vptr[tv[a] + 1]; ++k) row.push_back({vhandle[k], vphi[k]});
    std::sort(row.begin(), row.end(), [](const std::pair<int, double>& x, const std::pair<int, double>& y) {
      return x.first < y.first;
    });
    std::vector<std::pair<int, double>> merged;
    for (auto& pr : row) {
      if (!merged.empty() && merged.back().first == pr.first)
        merged.back().second += pr.second;
      else
        merged.push_back(pr);
    }
    for (auto& pr : merged) pr.second *= 0.25;
    row.swap(merged);
  }
  // partitions in ascending label order
  std::vector<int32_t> labels(part, part + T);
  std::sort(labels.begin(), labels.end());
  labels.erase(std::unique(labels.begin(), labels.end()), labels.end());
  std::vector<std::vector<int32_t>> ids(labels.size());
  for (int64_t t = 0; t < T; ++t) {
    const size_t p = size_t(std::lower_bound(labels.begin(), labels.end(), part[t]) - labels.begin());
    ids[p].push_back(int32_t(t));
  }
  std::vector<PartFit> fits(labels.size());
  const int ntask = int(labels.size());
  int nth = P.n_threads > 0 ? P.n_threads : int(std::max(1u, std::thread::hardware_concurrency()));
  nth = std::max(1, std::min(nth, ntask));
  std::atomic<int> next(0);
  std::vector<int> order(ntask);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return ids[a].size() > ids[b].size(); });
  std::vector<std::thread> pool;
  for (int k = 0; k < nth; ++k)
    pool.emplace_back([&]() {
      for (int q = next++; q < ntask; q = next++) fits[order[q]] = fit_partition(ids[order[q]], vol, ev, labels[order[q]], P);
    });
  for (auto& th : pool) th.join();
  std::vector<std::pair<int32_t, double>> all;
  double worst = 0.0;
  for (auto& f : fits) {
    for (size_t q = 0; q < f.tets.size(); ++q) all.push_back({f.tets[q], f.w[q]});
    worst = std::max(worst, f.rel);
  }
  std::sort(all.begin(), all.end());
  sel.resize(all.size());
  wts.resize(all.size());
  for (size_t q = 0; q < all.size(); ++q) sel[q] = all[q].first, wts[q] = all[q].second;
  if (max_rel) *max_rel = worst;
  return MS_OK;
}

// Device lists for the cubature coarse matrix given the selected tets, the
// installed basis and the Dirichlet set.  Stage 1 entries: (tet q, local
// vertex a, handle j) for every unpinned vertex a of a selected tet and
// every handle j carried by an unpinned vertex of that tet, with the
// (b, k_bj) contributions; then (v, j) for every unpinned vertex and each of
// its handles (mass, barrier and friction curvature).  Stage 2: per coarse
// pair (i <= j), the (k_vi, z) products.
ms_status build_cubature_lists(ms_ctx* c) {
  Cubature& C = c->cub;
  const Basis& B = c->basis;
  const int64_t n = c->n;
  std::vector<uint8_t> pinned(n, 0);
  for (int v : c->h_dbc) pinned[v] = 1;
  std::vector<int4> info;
  std::vector<double> scale;
  std::vector<int32_t> ent;
  std::vector<int32_t> zv, zh;  // vertex and handle of each stage-1 row (for stage 2)
  for (size_t q = 0; q < C.tets.size(); ++q) {
    const int32_t t = C.tets[q];
    const int32_t* tv = c->h_tets.data() + 4 * int64_t(t);
    std::vector<int> hs;
    for (int a = 0; a < 4; ++a)
      if (!pinned[tv[a]])
        for (int64_t k = B.vptr[tv[a]]; k < B.vptr[tv[a] + 1]; ++k) hs.push_back(B.vhandle[k]);
    std::sort(hs.begin(), hs.end());
    hs.erase(std::unique(hs.begin(), hs.end()), hs.end());
    const double s = C.w[q] / c->h_vol[t];
    for (int a = 0; a < 4; ++a) {
      if (pinned[tv[a]]) continue;
      for (int j : hs) {
        const int first = int(ent.size() / 2);
        for (int b = 0; b < 4; ++b) {
          if (pinned[tv[b]]) continue;
          for (int64_t k = B.vptr[tv[b]]; k < B.vptr[tv[b] + 1]; ++k)
            if (B.vhandle[k] == j) {
              ent.push_back(b);
              ent.push_back(int32_t(k));
            }
        }
        info.push_back(make_int4(t, a, first, int(ent.size() / 2)));
        scale.push_back(s);
        zv.push_back(tv[a]);
        zh.push_back(j);
      }
    }
  }
  for (int64_t v = 0; v < n; ++v) {
    if (pinned[v]) continue;
    for (int64_t k = B.vptr[v]; k < B.vptr[v + 1]; ++k) {
      info.push_back(make_int4(-1 - int32_t(v), int32_t(k), 0, 0));
      scale.push_back(0.0);
      zv.push_back(int32_t(v));
      zh.push_back(B.vhandle[k]);
    }
  }
  const int64_t nz = int64_t(info.size());
  if (nz >= (int64_t(1) << 31) || ent.size() >= (size_t(1) << 31)) return fail(c, MS_E_ARG, "cubature too large");
  // stage 2: for every row (v, j) and every handle i <= j on v, the product
  // phi_vi (x) Z_(v,j) belongs to pair (i, j)
  const int64_t m = B.m;
  std::unordered_map<int64_t, int32_t> pid;
  std::vector<std::pair<int, int>> pairs;
  std::vector<std::vector<std::pair<int, int>>> lists;
  for (int64_t z = 0; z < nz; ++z) {
    const int v = zv[z], j = zh[z];
    for (int64_t k = B.vptr[v]; k < B.vptr[v + 1]; ++k) {
      const int i = B.vhandle[k];
      if (i > j) continue;
      auto ins = pid.emplace(int64_t(i) * m + j, int32_t(pairs.size()));
      if (ins.second) {
        pairs.push_back({i, j});
        lists.emplace_back();
      }
      lists[ins.first->second].push_back({int(k), int(z)});
    }
  }
  std::vector<int> order(pairs.size());
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return pairs[a] < pairs[b]; });
  std::vector<int32_t> pair_ij, pptr(1, 0), pent;
  for (int id : order) {
    pair_ij.push_back(pairs[id].first);
    pair_ij.push_back(pairs[id].second);
    for (auto& e : lists[id]) {
      pent.push_back(e.first);
      pent.push_back(e.second);
    }
    pptr.push_back(int32_t(pent.size() / 2));
  }
  for (void* p : {static_cast<void*>(C.d_info), static_cast<void*>(C.d_scale), static_cast<void*>(C.d_ent),
                  static_cast<void*>(C.d_Z), static_cast<void*>(C.d_pair_ij), static_cast<void*>(C.d_pair_ptr),
                  static_cast<void*>(C.d_pair_ent)})
    if (p) dfree(c, p);
  C.d_info = nullptr, C.d_scale = nullptr, C.d_ent = nullptr, C.d_Z = nullptr;
  C.d_pair_ij = C.d_pair_ptr = C.d_pair_ent = nullptr;
  ms_status s;
  if (ent.empty()) ent.assign(2, 0);
  if ((s = upload(c, &C.d_info, info.data(), std::max<size_t>(1, info.size()))) ||
      (s = upload(c, &C.d_scale, scale.data(), std::max<size_t>(1, scale.size()))) ||
      (s = upload(c, &C.d_ent, ent.data(), ent.size())) || (s = alloc_n(c, &C.d_Z, 36 * size_t(std::max<int64_t>(1, nz)))))
    return s;
  if (pent.empty()) pent.assign(2, 0);
  if (pair_ij.empty()) pair_ij.assign(2, 0);
  if ((s = upload(c, &C.d_pair_ij, pair_ij.data(), pair_ij.size())) ||
      (s = upload(c, &C.d_pair_ptr, pptr.data(), pptr.size())) ||
      (s = upload(c, &C.d_pair_ent, pent.data(), pent.size())))
    return s;
  C.nz = nz;
  C.npairs = int32_t(order.size());
  C.built = true;
  return MS_OK;
}

}  // namespace ms

using namespace ms;

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
struct ms_cubature {
  std::vector<int32_t> tets;
  std::vector<double> w;
  double max_rel = 0.0;
};

namespace {

ms_status check_params(double tol, int32_t n_init, int32_t n_add, int32_t max_rounds) {
  if (!(tol >= 0.0) || !std::isfinite(tol) || n_init < 1 || n_add < 1 || max_rounds < 0) return MS_E_ARG;
  return MS_OK;
}

}  // namespace

extern "C" {

ms_status ms_cubature_compute(int64_t n, const double* rest, int64_t T, const int32_t* tets, const int32_t* part,
                              int32_t m, const int64_t* vptr, const int32_t* vhandle, const double* vphi,
                              double tol, int32_t n_init, int32_t n_add, int32_t max_rounds, uint64_t seed,
                              int32_t n_threads, ms_cubature** out) {
  if (!rest || !tets || !part || !vptr || !out || n < 1 || T < 1 || m < 1) return MS_E_ARG;
  if (check_params(tol, n_init, n_add, max_rounds)) return MS_E_ARG;
  for (int64_t i = 0; i < 4 * T; ++i)
    if (tets[i] < 0 || tets[i] >= n) return MS_E_ARG;
  for (int64_t t = 0; t < T; ++t)
    if (part[t] < 0) return MS_E_ARG;
  if (vptr[0] != 0) return MS_E_ARG;
  for (int64_t v = 0; v < n; ++v)
    if (vptr[v + 1] < vptr[v]) return MS_E_ARG;
  if (vptr[n] > 0 && (!vhandle || !vphi)) return MS_E_ARG;
  for (int64_t k = 0; k < vptr[n]; ++k)
    if (vhandle[k] < 0 || vhandle[k] >= m || !std::isfinite(vphi[k])) return MS_E_ARG;
  CubatureParams P{tol, n_init, n_add, max_rounds, seed, n_threads};
  ms_cubature* r = new ms_cubature();
  ms_status s = fit_cubature_host(n, rest, T, tets, part, vptr, vhandle, vphi, P, r->tets, r->w, &r->max_rel);
  if (s) {
    delete r;
    return s;
  }
  *out = r;
  return MS_OK;
}

ms_status ms_cubature_get(const ms_cubature* q, int64_t* n_pts, int32_t* tets, double* weights,
                          double* max_rel_residual) {
  if (!q || !n_pts) return MS_E_ARG;
  *n_pts = int64_t(q->tets.size());
  if (tets) std::copy(q->tets.begin(), q->tets.end(), tets);
  if (weights) std::copy(q->w.begin(), q->w.end(), weights);
  if (max_rel_residual) *max_rel_residual = q->max_rel;
  return MS_OK;
}

void ms_cubature_free(ms_cubature* q) { delete q; }

ms_status ms_set_cubature(ms_ctx* c, int64_t n_pts, const int32_t* tets, const double* weights) {
  if (!c) return MS_E_ARG;
  if (c->stage < 2) return fail(c, MS_E_ORDER, "upload mesh and material first");
  if (n_pts < 0 || (n_pts > 0 && (!tets || !weights))) return fail(c, MS_E_ARG, "bad cubature arrays");
  std::vector<std::pair<int32_t, double>> all(n_pts);
  for (int64_t q = 0; q < n_pts; ++q) {
    if (tets[q] < 0 || tets[q] >= c->T) return fail(c, MS_E_ARG, "cubature tet out of range");
    if (!(weights[q] >= 0.0) || !std::isfinite(weights[q])) return fail(c, MS_E_ARG, "bad cubature weight");
    all[q] = {tets[q], weights[q]};
  }
  std::sort(all.begin(), all.end());
  for (int64_t q = 1; q < n_pts; ++q)
    if (all[q].first == all[q - 1].first) return fail(c, MS_E_ARG, "repeated cubature tet");
  c->cub.tets.resize(n_pts);
  c->cub.w.resize(n_pts);
  for (int64_t q = 0; q < n_pts; ++q) c->cub.tets[q] = all[q].first, c->cub.w[q] = all[q].second;
  c->cub.present = n_pts > 0;
  c->cub.built = false;
  c->coarse_valid = 0;
  if (!c->cub.present) c->coarse_mode = MS_COARSE_EXACT;
  return MS_OK;
}

ms_status ms_build_cubature(ms_ctx* c, double tol, int32_t n_init, int32_t n_add, int32_t max_rounds,
                            uint64_t seed, double* max_rel_residual) {
  if (!c) return MS_E_ARG;
  if (!c->has_basis) return fail(c, MS_E_ORDER, "build or set a basis first");
  if (check_params(tol, n_init, n_add, max_rounds)) return fail(c, MS_E_ARG, "bad cubature parameters");
  const Basis& B = c->basis;
  if (int64_t(B.part.size()) != c->T) return fail(c, MS_E_ORDER, "the basis has no partitioning (ms_set_basis)");
  for (int32_t p : B.part)
    if (p < 0) return fail(c, MS_E_ORDER, "the basis has no partitioning (ms_set_basis)");
  CubatureParams P{tol, n_init, n_add, max_rounds, seed, 0};
  std::vector<int32_t> sel;
  std::vector<double> w;
  ms_status s = fit_cubature_host(c->n, c->h_rest.data(), c->T, c->h_tets.data(), B.part.data(), B.vptr.data(),
                                  B.vhandle.data(), B.vphi.data(), P, sel, w, max_rel_residual);
  if (s) return fail(c, s, "cubature fit failed");
  return ms_set_cubature(c, int64_t(sel.size()), sel.data(), w.data());
}

ms_status ms_get_cubature(const ms_ctx* c, int64_t* n_pts, int32_t* tets, double* weights) {
  if (!c || !n_pts) return MS_E_ARG;
  *n_pts = int64_t(c->cub.tets.size());
  if (tets) std::copy(c->cub.tets.begin(), c->cub.tets.end(), tets);
  if (weights) std::copy(c->cub.w.begin(), c->cub.w.end(), weights);
  return MS_OK;
}

ms_status ms_set_coarse_integration(ms_ctx* c, int32_t mode) {
  if (!c) return MS_E_ARG;
  if (mode != MS_COARSE_EXACT && mode != MS_COARSE_CUBATURE) return fail(c, MS_E_ARG, "bad coarse integration mode");
  if (mode == MS_COARSE_CUBATURE && !c->cub.present) return fail(c, MS_E_ORDER, "no cubature installed");
  if (c->coarse_mode != mode) c->coarse_valid = 0;
  c->coarse_mode = mode;
  return MS_OK;
}

}  // extern "C"
