// Cluster tree and block lists (host).  KD binary space partition of the
// parameter points (Sec. 4.2: KD-tree node ordering with leaf clusters of
// size m) and the strong-admissibility partition of the H2 format (Sec. 2 and
// Sec. 3.1: a block is low rank when its clusters are far apart relative to
// their size; dense blocks only at the leaf level).  Compiled without
// floating-point contraction so that every comparison is decided by plain
// IEEE operations in a fixed order.
#include <algorithm>
#include <numeric>

#include "internal.h"

namespace h2 {

static bool admissible(const h2_tree* t, int l, int a, int b) {
  const int d = t->dim;
  const double* la = &t->lo[l][(size_t)a * d];
  const double* ha = &t->hi[l][(size_t)a * d];
  const double* lb = &t->lo[l][(size_t)b * d];
  const double* hb = &t->hi[l][(size_t)b * d];
  const double eta2 = t->eta * t->eta;
  double da = 0.0, db = 0.0, dist = 0.0;
  for (int k = 0; k < d; ++k) {
    double ea = ha[k] - la[k];
    double eb = hb[k] - lb[k];
    double g = std::max(0.0, std::max(lb[k] - ha[k], la[k] - hb[k]));
    double ea2 = ea * ea, eb2 = eb * eb, g2 = g * g;
    da = da + ea2;
    db = db + eb2;
    dist = dist + g2;
  }
  double prod = eta2 * dist;
  return std::max(da, db) <= prod;
}

void tree_build(h2_tree* t) {
  const int n = t->n, d = t->dim, m = t->leaf;
  int L = 0;
  while ((int64_t(m) << L) < n) ++L;
  t->L = L;
  std::vector<std::vector<int64_t>> clusters(1);
  clusters[0].resize(n);
  std::iota(clusters[0].begin(), clusters[0].end(), 0);
  t->lo.assign(L + 1, {});
  t->hi.assign(L + 1, {});
  t->offsets.assign(L + 1, {});
  const double* P = t->points.data();
  for (int l = 0; l <= L; ++l) {
    const int nc = (int)clusters.size();
    t->lo[l].assign((size_t)nc * d, 0.0);
    t->hi[l].assign((size_t)nc * d, 0.0);
    t->offsets[l].assign(nc + 1, 0);
    for (int c = 0; c < nc; ++c) {
      const auto& idx = clusters[c];
      for (int k = 0; k < d; ++k) {
        double lo = P[idx[0] * d + k], hi = lo;
        for (int64_t u : idx) {
          lo = std::min(lo, P[u * d + k]);
          hi = std::max(hi, P[u * d + k]);
        }
        t->lo[l][(size_t)c * d + k] = lo;
        t->hi[l][(size_t)c * d + k] = hi;
      }
      t->offsets[l][c + 1] = t->offsets[l][c] + (int64_t)idx.size();
    }
    if (l == L) break;
    std::vector<std::vector<int64_t>> next;
    next.reserve(2 * nc);
    for (int c = 0; c < nc; ++c) {
      auto idx = clusters[c];
      int dim = 0;
      double best = t->hi[l][(size_t)c * d] - t->lo[l][(size_t)c * d];
      for (int k = 1; k < d; ++k) {
        double e = t->hi[l][(size_t)c * d + k] - t->lo[l][(size_t)c * d + k];
        if (e > best) { best = e; dim = k; }
      }
      std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        double xa = P[a * d + dim], xb = P[b * d + dim];
        if (xa != xb) return xa < xb;
        return a < b;
      });
      size_t half = (idx.size() + 1) / 2;
      next.emplace_back(idx.begin(), idx.begin() + half);
      next.emplace_back(idx.begin() + half, idx.end());
    }
    clusters.swap(next);
  }
  t->perm.clear();
  t->perm.reserve(n);
  for (auto& c : clusters) t->perm.insert(t->perm.end(), c.begin(), c.end());

  // dual traversal from (root, root)
  t->far.assign(L + 1, {});
  t->near.clear();
  std::vector<std::pair<int, int>> cand{{0, 0}};
  for (int l = 0; l <= L; ++l) {
    std::vector<std::pair<int, int>> nxt;
    for (auto [a, b] : cand) {
      if (l >= 1 && admissible(t, l, a, b)) {
        t->far[l].push_back({a, b});
      } else if (l == L) {
        t->near.push_back({a, b});
      } else {
        for (int x = 2 * a; x <= 2 * a + 1; ++x)
          for (int y = 2 * b; y <= 2 * b + 1; ++y) nxt.push_back({x, y});
      }
    }
    cand.swap(nxt);
  }
  for (auto& f : t->far) std::sort(f.begin(), f.end());
  std::sort(t->near.begin(), t->near.end());

  // flattened cluster data and CSR lists
  const int ncl = t->nclusters();
  t->cstart.assign(ncl, 0);
  t->csize.assign(ncl, 0);
  for (int l = 0; l <= L; ++l)
    for (int i = 0; i < (1 << l); ++i) {
      t->cstart[cid(l, i)] = (int32_t)t->offsets[l][i];
      t->csize[cid(l, i)] = (int32_t)(t->offsets[l][i + 1] - t->offsets[l][i]);
    }
  t->max_leaf = 0;
  for (int i = 0; i < (1 << L); ++i) t->max_leaf = std::max(t->max_leaf, t->csize[cid(L, i)]);
  t->far_ptr.clear();
  t->far_col.clear();
  t->far_ptr_base.assign(L + 2, 0);
  t->far_base.assign(L + 2, 0);
  for (int l = 0; l <= L; ++l) {
    t->far_ptr_base[l] = (int64_t)t->far_ptr.size();
    t->far_base[l] = (int64_t)t->far_col.size();
    std::vector<int32_t> cnt((1 << l) + 1, 0);
    for (auto [a, b] : t->far[l]) cnt[a + 1]++;
    for (int i = 0; i < (1 << l); ++i) cnt[i + 1] += cnt[i];
    // pointers are global indices into far_col
    for (auto& c : cnt) c += (int32_t)t->far_base[l];
    t->far_ptr.insert(t->far_ptr.end(), cnt.begin(), cnt.end());
    for (auto [a, b] : t->far[l]) t->far_col.push_back(b);
  }
  t->far_ptr_base[L + 1] = (int64_t)t->far_ptr.size();
  t->far_base[L + 1] = (int64_t)t->far_col.size();
  t->near_ptr.assign((1 << L) + 1, 0);
  t->near_col.clear();
  for (auto [a, b] : t->near) t->near_ptr[a + 1]++;
  for (int i = 0; i < (1 << L); ++i) t->near_ptr[i + 1] += t->near_ptr[i];
  for (auto [a, b] : t->near) t->near_col.push_back(b);

}

void tree_device(const h2_tree* tc) {
  h2_tree* t = const_cast<h2_tree*>(tc);
  if (t->device_ready) return;
  std::vector<int32_t> perm32(t->perm.begin(), t->perm.end());
  upload(t->d_perm, perm32);
  upload(t->d_cstart, t->cstart);
  upload(t->d_csize, t->csize);
  upload(t->d_far_ptr, t->far_ptr);
  upload(t->d_far_col, t->far_col);
  upload(t->d_near_ptr, t->near_ptr);
  upload(t->d_near_col, t->near_col);
  t->device_ready = true;
}

}  // namespace h2
