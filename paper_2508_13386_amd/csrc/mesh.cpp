// Host-side precompute for an uploaded tet mesh: rest shape matrices,
// volumes, vertex-tet incidence, the block-sparse Hessian pattern in the
// sliced BSR3 layout, and the gather lists that let the assembly kernels sum
// element blocks into Hessian slots and element gradients into vertices
// without atomics and in a fixed order (so results are bitwise reproducible).
#include <algorithm>
#include <cstring>
#include <cmath>
#include <cstdlib>
#include <numeric>

#include "ms_internal.h"

namespace ms {

// Local pair index of the 10 stored element blocks (a <= b).
static inline int pair_index(int a, int b) {
  // (0,0)=0 (0,1)=1 (0,2)=2 (0,3)=3 (1,1)=4 (1,2)=5 (1,3)=6 (2,2)=7 (2,3)=8 (3,3)=9
  static const int tbl[4][4] = {{0, 1, 2, 3}, {1, 4, 5, 6}, {2, 5, 7, 8}, {3, 6, 8, 9}};
  return tbl[a][b];
}

ms_status mesh_geometry(ms_ctx* c) {
  const int64_t n = c->n, T = c->T;
  c->h_vol.assign(T, 0.0);
  c->h_Dminv.assign(9 * T, 0.0);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t* v = &c->h_tets[4 * t];
    double Dm[3][3];
    for (int col = 0; col < 3; ++col)
      for (int i = 0; i < 3; ++i) Dm[i][col] = c->h_rest[3 * v[col + 1] + i] - c->h_rest[3 * v[0] + i];
    double det = Dm[0][0] * (Dm[1][1] * Dm[2][2] - Dm[1][2] * Dm[2][1]) -
                 Dm[0][1] * (Dm[1][0] * Dm[2][2] - Dm[1][2] * Dm[2][0]) +
                 Dm[0][2] * (Dm[1][0] * Dm[2][1] - Dm[1][1] * Dm[2][0]);
    if (!(det > 0.0) || !std::isfinite(det))
      return fail(c, MS_E_MESH, "rest tet " + std::to_string(t) + " has non-positive volume");
    double inv = 1.0 / det;
    double* m = &c->h_Dminv[9 * t];
    m[0] = (Dm[1][1] * Dm[2][2] - Dm[1][2] * Dm[2][1]) * inv;
    m[1] = (Dm[0][2] * Dm[2][1] - Dm[0][1] * Dm[2][2]) * inv;
    m[2] = (Dm[0][1] * Dm[1][2] - Dm[0][2] * Dm[1][1]) * inv;
    m[3] = (Dm[1][2] * Dm[2][0] - Dm[1][0] * Dm[2][2]) * inv;
    m[4] = (Dm[0][0] * Dm[2][2] - Dm[0][2] * Dm[2][0]) * inv;
    m[5] = (Dm[0][2] * Dm[1][0] - Dm[0][0] * Dm[1][2]) * inv;
    m[6] = (Dm[1][0] * Dm[2][1] - Dm[1][1] * Dm[2][0]) * inv;
    m[7] = (Dm[0][1] * Dm[2][0] - Dm[0][0] * Dm[2][1]) * inv;
    m[8] = (Dm[0][0] * Dm[1][1] - Dm[0][1] * Dm[1][0]) * inv;
    c->h_vol[t] = det / 6.0;
  }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < n; ++v)
    for (int i = 0; i < 3; ++i) {
      lo[i] = std::min(lo[i], c->h_rest[3 * v + i]);
      hi[i] = std::max(hi[i], c->h_rest[3 * v + i]);
    }
  c->bbox_diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                           (hi[2] - lo[2]) * (hi[2] - lo[2]));
  return MS_OK;
}

ms_status build_mesh(ms_ctx* c) {
  const int64_t n = c->n, T = c->T;
  ms_status s0 = mesh_geometry(c);
  if (s0) return s0;
  // vertex -> (tet, local) incidence, ordered by tet index
  std::vector<int32_t> vt_ptr(n + 1, 0), vt_code(4 * T);
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a) vt_ptr[c->h_tets[4 * t + a] + 1]++;
  for (int64_t v = 0; v < n; ++v) vt_ptr[v + 1] += vt_ptr[v];
  {
    std::vector<int32_t> fill(vt_ptr.begin(), vt_ptr.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a) vt_code[fill[c->h_tets[4 * t + a]]++] = int32_t(4 * t + a);
  }
  ms_status s;
  if ((s = upload(c, &c->d_rest, c->h_rest.data(), 3 * n))) return s;
  if ((s = upload(c, &c->d_tets, c->h_tets.data(), 4 * T))) return s;
  if ((s = upload(c, &c->d_Dminv, c->h_Dminv.data(), 9 * T))) return s;
  if ((s = upload(c, &c->d_vol, c->h_vol.data(), T))) return s;
  if ((s = upload(c, &c->d_vt_ptr, vt_ptr.data(), n + 1))) return s;
  if ((s = upload(c, &c->d_vt_code, vt_code.data(), 4 * T))) return s;
  return build_pattern(c);
}

void slice_layout(int64_t n, const int32_t* row_ptr, int S, std::vector<int32_t>& slice_base, int& maxw) {
  const int64_t ns = (n + S - 1) / S;
  slice_base.assign(ns + 1, 0);
  maxw = 0;
  for (int64_t s = 0; s < ns; ++s) {
    int32_t w = 0;
    for (int64_t r = s * S; r < std::min<int64_t>(n, (s + 1) * S); ++r) w = std::max(w, row_ptr[r + 1] - row_ptr[r]);
    slice_base[s + 1] = slice_base[s] + w * S;
    maxw = std::max(maxw, int(w));
  }
}

ms_status build_pattern(ms_ctx* c) {
  const int64_t n = c->n, T = c->T;
  Pattern& P = c->pat;
  P.n = n;
  c->agg.built = false;  // its block slots follow the pattern
  // adjacency (including self), sorted per row
  std::vector<std::vector<int32_t>> adj(n);
  for (int64_t v = 0; v < n; ++v) adj[v].push_back(int32_t(v));
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        if (a != b) adj[c->h_tets[4 * t + a]].push_back(c->h_tets[4 * t + b]);
  P.h_row_ptr.assign(n + 1, 0);
  for (int64_t v = 0; v < n; ++v) {
    auto& a = adj[v];
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
    P.h_row_ptr[v + 1] = P.h_row_ptr[v] + int32_t(a.size());
  }
  P.nnzb = P.h_row_ptr[n];
  P.h_col.resize(P.nnzb);
  for (int64_t v = 0; v < n; ++v) std::copy(adj[v].begin(), adj[v].end(), P.h_col.begin() + P.h_row_ptr[v]);
  // slice height: 32 rows per slice (two lanes per row), or MS_SLICE = 16,
  // 32 or 64; MS_SLICE = auto times the three layouts on this pattern (FP64
  // SpMV with constant values, interleaved rounds, best round kept) and keeps
  // 32 unless another is at least 3% faster.  The default is fixed so that
  // runs and profiles of one mesh use the same kernel instance.
  int S = 32;
  const char* env = std::getenv("MS_SLICE");
  if (env && std::strcmp(env, "auto") != 0) {
    const int want = std::atoi(env);
    if (want == 16 || want == 32 || want == 64) S = want;
  }
  if (env && std::strcmp(env, "auto") == 0) {
    const int cands[3] = {16, 32, 64};
    int32_t *d_sb[3] = {nullptr, nullptr, nullptr}, *d_sc[3] = {nullptr, nullptr, nullptr};
    int64_t ns[3], nsl[3];
    double best[3] = {1e300, 1e300, 1e300};
    ms_status st = MS_OK;
    for (int q = 0; q < 3 && !st; ++q) {
      const int cand = cands[q];
      std::vector<int32_t> sb;
      int mw = 0;
      slice_layout(n, P.h_row_ptr.data(), cand, sb, mw);
      ns[q] = int64_t(sb.size()) - 1;
      nsl[q] = sb.back();
      std::vector<int32_t> sc(nsl[q], -1);
      for (int64_t r = 0; r < n; ++r)
        for (int32_t k = 0; k < P.h_row_ptr[r + 1] - P.h_row_ptr[r]; ++k)
          sc[sb[r / cand] + int64_t(k) * cand + r % cand] = P.h_col[P.h_row_ptr[r] + k];
      if (!(st = upload(c, &d_sb[q], sb.data(), sb.size()))) st = upload(c, &d_sc[q], sc.data(), sc.size());
    }
    for (int round = 0; round < 5 && !st; ++round)
      for (int q = 0; q < 3 && !st; ++q) {
        const double t = time_spmv_layout(c, cands[q], d_sb[q], d_sc[q], ns[q], nsl[q], 10);
        if (t < 0) st = fail(c, MS_E_DEVICE, "SpMV layout timing failed");
        best[q] = std::min(best[q], t);
      }
    for (int q = 0; q < 3; ++q) {
      dfree(c, d_sb[q]);
      dfree(c, d_sc[q]);
    }
    if (st) return st;
    S = 32;
    double bt = best[1];
    for (int q : {0, 2})
      if (best[q] < 0.97 * best[1] && best[q] < bt) bt = best[q], S = cands[q];
  }
  P.S = S;
  // self-contact reserves `spare` extra block columns in every surface row
  // (contact slots, column -1 until a contact pair couples the row)
  std::vector<int32_t> lay_ptr(P.h_row_ptr);
  SelfContact& SC = c->sc;
  SC.h_spare0.assign(n, -1);
  if (SC.spare > 0) {
    std::vector<uint8_t> surf(n, 0);
    for (int32_t v : SC.h_verts) surf[v] = 1;
    for (int64_t r = 0; r < n; ++r) {
      const int32_t len = P.h_row_ptr[r + 1] - P.h_row_ptr[r];
      if (surf[r]) SC.h_spare0[r] = len;
      lay_ptr[r + 1] = lay_ptr[r] + len + (surf[r] ? SC.spare : 0);
    }
  }
  slice_layout(n, lay_ptr.data(), S, P.h_slice_base, P.maxw);
  P.nslices = int64_t(P.h_slice_base.size()) - 1;
  P.nslots = P.h_slice_base[P.nslices];
  std::vector<int32_t> scol(P.nslots, -1), diag_slot(n);
  P.h_slot_of_bsr.resize(P.nnzb);
  for (int64_t r = 0; r < n; ++r) {
    int64_t s = r / S, lane = r % S;
    for (int32_t k = 0; k < P.h_row_ptr[r + 1] - P.h_row_ptr[r]; ++k) {
      int64_t slot = P.h_slice_base[s] + int64_t(k) * S + lane;
      int32_t col = P.h_col[P.h_row_ptr[r] + k];
      scol[slot] = col;
      P.h_slot_of_bsr[P.h_row_ptr[r] + k] = slot;
      if (col == r) diag_slot[r] = int32_t(slot);
    }
  }
  // gather lists: every tet contributes block (a,b) to row tets[a], column tets[b]
  auto find_slot = [&](int32_t i, int32_t j) -> int64_t {
    const int32_t* b = &P.h_col[P.h_row_ptr[i]];
    const int32_t* e = &P.h_col[P.h_row_ptr[i + 1]];
    int64_t k = std::lower_bound(b, e, j) - b;
    return P.h_slice_base[i / S] + k * S + (i % S);
  };
  std::vector<int32_t> gcnt(P.nslots + 1, 0);
  std::vector<int64_t> tslot(16 * T);
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int64_t sl = find_slot(c->h_tets[4 * t + a], c->h_tets[4 * t + b]);
        tslot[16 * t + 4 * a + b] = sl;
        gcnt[sl + 1]++;
      }
  for (int64_t s = 0; s < P.nslots; ++s) gcnt[s + 1] += gcnt[s];
  std::vector<int32_t> gcode(16 * T);
  {
    std::vector<int32_t> fill(gcnt.begin(), gcnt.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          int64_t sl = tslot[16 * t + 4 * a + b];
          int pr = pair_index(std::min(a, b), std::max(a, b));
          int tr = a > b ? 1 : 0;
          gcode[fill[sl]++] = int32_t((t * 10 + pr) * 2 + tr);
        }
  }
  ms_status s;
  if (SC.spare > 0) SC.h_col = scol;
  if ((s = upload(c, &P.d_slice_base, P.h_slice_base.data(), P.nslices + 1))) return s;
  if ((s = upload(c, &P.d_col, scol.data(), P.nslots))) return s;
  if ((s = upload(c, &P.d_diag_slot, diag_slot.data(), n))) return s;
  if ((s = upload(c, &c->d_gptr, gcnt.data(), P.nslots + 1))) return s;
  if ((s = upload(c, &c->d_gcode, gcode.data(), 16 * T))) return s;
  return MS_OK;
}

}  // namespace ms
