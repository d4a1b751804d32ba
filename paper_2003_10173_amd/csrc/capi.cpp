// extern "C" entry points for trees, matrices and HGEMV.  Every entry point
// converts internal exceptions into an h2_status and records the message.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#include "internal.h"
#include "vecops.h"

namespace h2 {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("H2_VERBOSE");
    return e && e[0] == '1';
  }();
  return v;
}

template <class F>
static h2_status guarded(F&& f) {
  try {
    f();
    return H2_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return H2_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return H2_EINVAL;
  }
}

h2_status guarded_status(const std::function<void()>& f) { return guarded(f); }

void matrix_copy_convert(const h2_matrix* A, h2_matrix* B, double scale, hipStream_t s);
void matrix_identity(h2_matrix* A, const h2_tree* t, double alpha, hipStream_t s);

}  // namespace h2

using namespace h2;

extern "C" {

const char* h2_status_string(h2_status s) {
  switch (s) {
    case H2_OK: return "ok";
    case H2_EINVAL: return "invalid argument";
    case H2_ENOMEM: return "out of memory";
    case H2_EDEVICE: return "device error";
    case H2_ECALLBACK: return "sampler callback failed";
    case H2_ENUMERIC: return "non-finite values";
    case H2_ENOTCONVERGED: return "not converged";
    case H2_EDIVERGED: return "diverged";
  }
  return "unknown status";
}

const char* h2_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ tree
h2_status h2_tree_create(const double* points_host, int n, int dim, int leaf_size, double eta,
                         h2_tree** out) {
  return guarded([&] {
    H2_CHECK(out && points_host, H2_EINVAL, "null argument");
    H2_CHECK(n >= 1 && dim >= 1 && dim <= 3, H2_EINVAL, "need n >= 1 and 1 <= dim <= 3");
    H2_CHECK(leaf_size >= 1 && leaf_size <= 64, H2_EINVAL, "leaf_size must be in 1..64");
    H2_CHECK(eta > 0, H2_EINVAL, "eta must be positive");
    for (int64_t i = 0; i < (int64_t)n * dim; ++i)
      H2_CHECK(std::isfinite(points_host[i]), H2_EINVAL, "non-finite point coordinate");
    auto t = std::make_unique<h2_tree>();
    t->n = n;
    t->dim = dim;
    t->leaf = leaf_size;
    t->eta = eta;
    t->points.assign(points_host, points_host + (size_t)n * dim);
    tree_build(t.get());
    H2_CHECK(t->L < H2_MAX_LEVELS - 1, H2_EINVAL, "too many levels");
    *out = t.release();
  });
}

void h2_tree_destroy(h2_tree* tree) { delete tree; }

h2_status h2_tree_info(const h2_tree* t, int* n, int* levels, int* leaf_size, int* dim) {
  return guarded([&] {
    H2_CHECK(t, H2_EINVAL, "null tree");
    if (n) *n = t->n;
    if (levels) *levels = t->L;
    if (leaf_size) *leaf_size = t->leaf;
    if (dim) *dim = t->dim;
  });
}

h2_status h2_tree_perm(const h2_tree* t, int64_t* perm) {
  return guarded([&] {
    H2_CHECK(t && perm, H2_EINVAL, "null argument");
    std::copy(t->perm.begin(), t->perm.end(), perm);
  });
}

h2_status h2_tree_offsets(const h2_tree* t, int level, int64_t* off) {
  return guarded([&] {
    H2_CHECK(t && off, H2_EINVAL, "null argument");
    H2_CHECK(level >= 0 && level <= t->L, H2_EINVAL, "level out of range");
    std::copy(t->offsets[level].begin(), t->offsets[level].end(), off);
  });
}

h2_status h2_tree_pair_count(const h2_tree* t, int level, int64_t* count) {
  return guarded([&] {
    H2_CHECK(t && count, H2_EINVAL, "null argument");
    H2_CHECK(level >= -1 && level <= t->L, H2_EINVAL, "level out of range");
    *count = level < 0 ? (int64_t)t->near.size() : (int64_t)t->far[level].size();
  });
}

h2_status h2_tree_pairs(const h2_tree* t, int level, int32_t* pairs) {
  return guarded([&] {
    H2_CHECK(t && pairs, H2_EINVAL, "null argument");
    H2_CHECK(level >= -1 && level <= t->L, H2_EINVAL, "level out of range");
    const auto& v = level < 0 ? t->near : t->far[level];
    for (size_t i = 0; i < v.size(); ++i) {
      pairs[2 * i] = v[i].first;
      pairs[2 * i + 1] = v[i].second;
    }
  });
}

// ------------------------------------------------------------------ matrices
h2_status h2_matrix_sizes(const h2_tree* t, const int32_t* ranks, int64_t* nU, int64_t* nE,
                          int64_t* nS, int64_t* nD) {
  return guarded([&] {
    H2_CHECK(t && ranks, H2_EINVAL, "null argument");
    std::vector<int32_t> r(ranks, ranks + t->nclusters());
    const int L = t->L;
    int64_t u = 0, e = 0, s = 0, d = 0;
    for (int i = 0; i < (1 << L); ++i) u += (int64_t)t->csize[cid(L, i)] * r[cid(L, i)];
    r[0] = 0;  // the root carries no basis
    for (int c = 1; c < t->nclusters(); ++c) e += (int64_t)r[c] * r[(c - 1) / 2];
    for (int l = 1; l <= L; ++l)
      for (auto [a, b] : t->far[l]) s += (int64_t)r[cid(l, a)] * r[cid(l, b)];
    for (auto [a, b] : t->near) d += (int64_t)t->csize[cid(L, a)] * t->csize[cid(L, b)];
    if (nU) *nU = u;
    if (nE) *nE = e;
    if (nS) *nS = s;
    if (nD) *nD = d;
  });
}

h2_status h2_matrix_import(const h2_tree* t, const int32_t* ranks, const double* U,
                           const double* E, const double* S, const double* D, h2_matrix** out) {
  return guarded([&] {
    H2_CHECK(t && ranks && out && D, H2_EINVAL, "null argument");
    auto A = std::make_unique<h2_matrix>();
    std::vector<int32_t> r(ranks, ranks + t->nclusters());
    for (auto k : r) H2_CHECK(k >= 0 && k <= 4096, H2_EINVAL, "rank out of range");
    matrix_layout(A.get(), t, r);
    matrix_alloc(A.get(), H2_FP64);
    auto put = [&](DevBuf& b, const double* h, int64_t n) {
      if (n > 0) {
        H2_CHECK(h != nullptr, H2_EINVAL, "missing block array");
        H2_HIP(hipMemcpy(b.p, h, n * sizeof(double), hipMemcpyHostToDevice));
      }
    };
    put(A->st.U, U, A->nU());
    put(A->st.E, E, A->nE());
    put(A->st.S, S, A->nS());
    put(A->st.D, D, A->nD());
    *out = A.release();
  });
}

h2_status h2_matrix_ranks(const h2_matrix* A, int32_t* ranks) {
  return guarded([&] {
    H2_CHECK(A && ranks, H2_EINVAL, "null argument");
    std::copy(A->rank.begin(), A->rank.end(), ranks);
  });
}

h2_status h2_matrix_export(const h2_matrix* A, double* U, double* E, double* S, double* D) {
  return guarded([&] {
    H2_CHECK(A, H2_EINVAL, "null matrix");
    std::unique_ptr<h2_matrix> tmp;
    const h2_matrix* src = A;
    if (A->st.prec != H2_FP64) {
      tmp = matrix_clone_layout(A);
      matrix_alloc(tmp.get(), H2_FP64);
      matrix_copy_convert(A, tmp.get(), 1.0, 0);
      H2_HIP(hipDeviceSynchronize());
      src = tmp.get();
    }
    auto get = [&](double* h, const DevBuf& b, int64_t n) {
      if (h && n > 0) H2_HIP(hipMemcpy(h, b.p, n * sizeof(double), hipMemcpyDeviceToHost));
    };
    get(U, src->st.U, src->nU());
    get(E, src->st.E, src->nE());
    get(S, src->st.S, src->nS());
    get(D, src->st.D, src->nD());
  });
}

h2_status h2_matrix_words(const h2_matrix* A, int64_t* words, int64_t* bytes) {
  return guarded([&] {
    H2_CHECK(A, H2_EINVAL, "null matrix");
    const int64_t w = A->nU() + A->nE() + A->nS() + A->nD();
    if (words) *words = w;
    if (bytes) *bytes = w * (int64_t)A->st.elem();
  });
}

h2_status h2_matrix_convert(const h2_matrix* A, h2_precision prec, h2_matrix** out) {
  return guarded([&] {
    H2_CHECK(A && out, H2_EINVAL, "null argument");
    H2_CHECK(prec == H2_FP64 || prec == H2_FP32 || prec == H2_BF16, H2_EINVAL, "bad precision");
    auto B = matrix_clone_layout(A);
    matrix_alloc(B.get(), prec);
    matrix_copy_convert(A, B.get(), 1.0, 0);
    H2_HIP(hipDeviceSynchronize());
    *out = B.release();
  });
}

h2_status h2_matrix_scale(const h2_matrix* A, double alpha, h2_matrix** out) {
  return guarded([&] {
    H2_CHECK(A && out, H2_EINVAL, "null argument");
    auto B = matrix_clone_layout(A);
    matrix_alloc(B.get(), A->st.prec);
    matrix_copy_convert(A, B.get(), alpha, 0);
    H2_HIP(hipDeviceSynchronize());
    *out = B.release();
  });
}

h2_status h2_matrix_identity(const h2_tree* t, double alpha, h2_matrix** out) {
  return guarded([&] {
    H2_CHECK(t && out, H2_EINVAL, "null argument");
    auto A = std::make_unique<h2_matrix>();
    matrix_identity(A.get(), t, alpha, 0);
    H2_HIP(hipDeviceSynchronize());
    *out = A.release();
  });
}

void h2_destroy(h2_matrix* A) { delete A; }

// ------------------------------------------------------------------ HGEMV
h2_status h2_gemv(const h2_matrix* A, int nv, double alpha, const double* x, int ldx,
                  double beta, double* y, int ldy, hipStream_t s) {
  return guarded([&] {
    H2_CHECK(A, H2_EINVAL, "null matrix");
    const int n = A->tree->n;
    H2_CHECK(nv >= 0 && ldx >= n && ldy >= n, H2_EINVAL, "bad vector count or leading dimension");
    if (nv == 0) return;
    H2_CHECK(x && y, H2_EINVAL, "null vector");
    H2_CHECK(A->st.prec == H2_FP64, H2_EINVAL, "h2_gemv needs FP64 storage; use h2_gemv_f32");
    A->ws_vec.reserve((size_t)2 * n * nv * sizeof(double));
    double* xt = A->ws_vec.as<double>();
    double* yt = xt + (size_t)n * nv;
    gather_rows(A->tree, nv, x, ldx, xt, n, s);
    gemv_tree_f64(A, nv, 1.0, xt, n, 0.0, yt, n, s);
    scatter_rows(A->tree, nv, alpha, yt, n, beta, y, ldy, s);
  });
}

h2_status h2_gemv_f32(const h2_matrix* A, int nv, float alpha, const float* x, int ldx,
                      float beta, float* y, int ldy, hipStream_t s) {
  return guarded([&] {
    H2_CHECK(A, H2_EINVAL, "null matrix");
    const int n = A->tree->n;
    H2_CHECK(nv >= 0 && ldx >= n && ldy >= n, H2_EINVAL, "bad vector count or leading dimension");
    if (nv == 0) return;
    H2_CHECK(x && y, H2_EINVAL, "null vector");
    A->ws_vec.reserve((size_t)2 * n * nv * sizeof(float));
    float* xt = A->ws_vec.as<float>();
    float* yt = xt + (size_t)n * nv;
    gather_rows_f32(A->tree, nv, x, ldx, xt, n, s);
    gemv_tree_f32(A, nv, 1.0f, xt, n, 0.0f, yt, n, s);
    scatter_rows_f32(A->tree, nv, alpha, yt, n, beta, y, ldy, s);
  });
}

h2_status h2_norm2(const h2_matrix* A, int max_iter, double rel, uint64_t seed, hipStream_t s,
                   double* out) {
  return guarded([&] {
    H2_CHECK(A && out, H2_EINVAL, "null argument");
    H2_CHECK(A->st.prec == H2_FP64, H2_EINVAL, "h2_norm2 needs FP64 storage");
    auto op = [&](const double* v, double* w) { gemv_tree_f64(A, 1, 1.0, v, A->tree->n, 0.0, w, A->tree->n, s); };
    *out = power_norm_device(A->tree->n, op, seed, 0, rel <= 0 ? 1e-2 : rel, 3,
                             max_iter <= 0 ? 30 : max_iter, s, nullptr);
  });
}

}  // extern "C"
