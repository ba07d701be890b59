// Small host-side sparse symmetric positive definite solver used by the
// basis construction: reverse Cuthill-McKee ordering and an envelope
// (profile) Cholesky factorisation.  Matrices are given in full symmetric
// CSR form (both triangles).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <queue>
#include <vector>

namespace ms {

struct Csr {
  int n = 0;
  std::vector<int> ptr, idx;
  std::vector<double> val;
};

// Reverse Cuthill-McKee over the graph of A; returns perm[new] = old.
inline std::vector<int> rcm_order(const Csr& A) {
  const int n = A.n;
  std::vector<int> deg(n), perm;
  perm.reserve(n);
  for (int i = 0; i < n; ++i) deg[i] = A.ptr[i + 1] - A.ptr[i];
  std::vector<char> seen(n, 0);
  std::vector<int> nb;
  for (int start_scan = 0; start_scan < n; ++start_scan) {
    if (seen[start_scan]) continue;
    // pseudo-peripheral start: the last vertex reached by a BFS of this component
    int s = start_scan;
    {
      std::vector<int> comp;
      std::queue<int> q;
      q.push(s);
      comp.push_back(s);
      seen[s] = 2;
      while (!q.empty()) {
        int v = q.front();
        q.pop();
        for (int k = A.ptr[v]; k < A.ptr[v + 1]; ++k) {
          int w = A.idx[k];
          if (!seen[w]) {
            seen[w] = 2;
            comp.push_back(w);
            q.push(w);
          }
        }
      }
      s = comp.back();
      for (int v : comp) seen[v] = 0;
    }
    std::queue<int> q;
    q.push(s);
    seen[s] = 1;
    while (!q.empty()) {
      int v = q.front();
      q.pop();
      perm.push_back(v);
      nb.clear();
      for (int k = A.ptr[v]; k < A.ptr[v + 1]; ++k) {
        int w = A.idx[k];
        if (!seen[w]) {
          seen[w] = 1;
          nb.push_back(w);
        }
      }
      std::sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] < deg[b] || (deg[a] == deg[b] && a < b); });
      for (int w : nb) q.push(w);
    }
  }
  std::reverse(perm.begin(), perm.end());
  return perm;
}

// Envelope Cholesky A = L L^T of a permuted SPD matrix; row i of L is
// stored from its first structural non-zero column first[i] to i.
struct EnvelopeCholesky {
  int n = 0;
  std::vector<int> perm, iperm, first;
  std::vector<int64_t> start;  // offset of row i in val
  std::vector<double> val;
  int regularised = 0;

  bool factor(const Csr& A) {
    n = A.n;
    perm = rcm_order(A);
    iperm.assign(n, 0);
    for (int i = 0; i < n; ++i) iperm[perm[i]] = i;
    first.assign(n, 0);
    for (int i = 0; i < n; ++i) {
      int f = i;
      const int o = perm[i];
      for (int k = A.ptr[o]; k < A.ptr[o + 1]; ++k) f = std::min(f, iperm[A.idx[k]]);
      first[i] = f;
    }
    start.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) start[i + 1] = start[i] + (i - first[i] + 1);
    val.assign(start[n], 0.0);
    for (int i = 0; i < n; ++i) {
      const int o = perm[i];
      for (int k = A.ptr[o]; k < A.ptr[o + 1]; ++k) {
        const int j = iperm[A.idx[k]];
        if (j <= i) val[start[i] + (j - first[i])] += A.val[k];
      }
    }
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) dmax = std::max(dmax, std::fabs(val[start[i + 1] - 1]));
    for (int i = 0; i < n; ++i) {
      double* Li = &val[start[i]];
      const int fi = first[i];
      for (int j = fi; j < i; ++j) {
        const double* Lj = &val[start[j]];
        const int fj = first[j];
        const int k0 = std::max(fi, fj);
        double s = Li[j - fi];
        const double* a = Li + (k0 - fi);
        const double* b = Lj + (k0 - fj);
        for (int k = 0; k < j - k0; ++k) s -= a[k] * b[k];
        Li[j - fi] = s / Lj[j - fj];
      }
      double d = Li[i - fi];
      for (int k = 0; k < i - fi; ++k) d -= Li[k] * Li[k];
      if (!(d > 1e-14 * dmax)) {
        d = std::max(1e-14 * dmax, 1e-300);
        ++regularised;
      }
      Li[i - fi] = std::sqrt(d);
    }
    return true;
  }

  // Solves A x = b in place (b in original ordering).
  void solve(std::vector<double>& b) const {
    std::vector<double> y(n);
    for (int i = 0; i < n; ++i) y[i] = b[perm[i]];
    for (int i = 0; i < n; ++i) {
      const double* Li = &val[start[i]];
      const int fi = first[i];
      double s = y[i];
      for (int k = fi; k < i; ++k) s -= Li[k - fi] * y[k];
      y[i] = s / Li[i - fi];
    }
    for (int i = n - 1; i >= 0; --i) {
      const double* Li = &val[start[i]];
      const int fi = first[i];
      y[i] /= Li[i - fi];
      const double yi = y[i];
      for (int k = fi; k < i; ++k) y[k] -= Li[k - fi] * yi;
    }
    for (int i = 0; i < n; ++i) b[perm[i]] = y[i];
  }
};

}  // namespace ms
