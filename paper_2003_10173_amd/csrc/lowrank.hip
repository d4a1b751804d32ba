// Global low-rank pre-pass combined with the hierarchical construction
// (Sec. 3.3, the paragraph on combining the construction with global low-rank
// approximations): B B^T from the dense randomized range finder, the
// construction of the residual H - B B^T, and B B^T added back as a low-rank
// update by recompressing A_res + B B^T through the same construction.
//
// Range finder (Halko, Martinsson, Tropp, two passes): Y = H Omega with r + p
// Gaussian columns, Q from the QR of Y, T = Q^T (H Q) symmetrised, T = V
// diag(s) V^T by the Jacobi SVD (T is positive semi-definite), and the values
// above 1e-13 s_1 (at most r) give B = Q V_r diag(sqrt(s_r)).
#include <algorithm>
#include <cmath>
#include <functional>

#include "build.h"
#include "kernels_common.h"
#include "vecops.h"

namespace h2 {

h2_status guarded_status(const std::function<void()>& f);

namespace {

constexpr uint32_t PHASE_GLOBAL = 7;
constexpr double EIG_CUT = 1e-13;

// Gaussian block (n x ncols, ld n) keyed by tree row and column
__global__ void k_fill_gauss(uint64_t key, int n, int ncols, double* __restrict__ om) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * ncols) return;
  const int r = (int)(e % n), j = (int)(e / n);
  om[(size_t)j * n + r] = gauss_entry(key, (uint64_t)r, (uint64_t)j);
}

// y = inner(Omega) + sign * B (B^T Omega), tree order
struct LowRankCorrected : Sampler {
  Sampler* inner;
  const double* B;
  int n, k;
  double sign;
  DevBuf tmp;
  LowRankCorrected(Sampler* s, const double* b, int n_, int k_, double sg)
      : inner(s), B(b), n(n_), k(k_), sign(sg) {}
  void apply(Ctx& c, int ncols, const double* om, double* y) override {
    if (ncols <= 0) return;
    inner->apply(c, ncols, om, y);
    if (k > 0) {
      tmp.reserve((size_t)k * ncols * sizeof(double));
      double* W = tmp.as<double>();
      gemm_batched(c, {GemmDesc{B, om, W, k, ncols, n, n, n, k, 1, 0, 1.0, 0.0}});
      gemm_batched(c, {GemmDesc{B, W, y, n, ncols, k, n, k, n, 0, 0, sign, 1.0}});
    }
    applies += ncols;
  }
};

struct MatrixSampler : Sampler {
  const h2_matrix* A;
  explicit MatrixSampler(const h2_matrix* a) : A(a) {}
  void apply(Ctx& c, int ncols, const double* om, double* y) override {
    gemv_tree_f64(A, ncols, 1.0, om, A->tree->n, 0.0, y, A->tree->n, c.s);
    applies += ncols;
  }
};

}  // namespace

// B (n x k, tree order, ld n) into Bbuf; returns k
static int global_lowrank(const h2_tree* t, Sampler& S, int rank, int oversample, uint64_t seed,
                          Ctx& c, DevBuf& Bbuf) {
  const int n = t->n;
  const int b = std::min(rank + oversample, n);
  H2_CHECK(b >= 1 && b <= 1024, H2_EINVAL, "global rank + oversampling must be 1..1024");
  DevBuf om((size_t)n * b * sizeof(double)), y((size_t)n * b * sizeof(double));
  DevBuf q((size_t)n * b * sizeof(double)), z((size_t)n * b * sizeof(double));
  DevBuf tt((size_t)b * b * sizeof(double) * 2), sv((size_t)b * sizeof(double));
  DevBuf u((size_t)b * b * sizeof(double)), v((size_t)b * b * sizeof(double));
  DevBuf r((size_t)b * b * sizeof(double));
  const int64_t tot = (int64_t)n * b;
  k_fill_gauss<<<(unsigned)((tot + 255) / 256), 256, 0, c.s>>>(
      stream_key(seed, PHASE_GLOBAL, 0, 0, 0), n, b, om.as<double>());
  H2_LAUNCH_CHECK();
  S.apply(c, b, om.as<double>(), y.as<double>());
  // Q (n x b) from the QR of Y
  qr_auto(c, {QRDesc{y.as<double>(), n, n, b, q.as<double>(), n, r.as<double>(), b}});
  S.apply(c, b, q.as<double>(), z.as<double>());
  // T = Q^T Z, symmetrised: T <- (T + T^T) / 2
  double* T = tt.as<double>();
  double* Tt = T + (size_t)b * b;
  gemm_batched(c, {GemmDesc{q.as<double>(), z.as<double>(), T, b, b, n, n, n, b, 1, 0, 1.0, 0.0}});
  copy_batched(c, {CopyDesc{T, b, Tt, b, b, b, 1.0, 0.0, 1}});
  copy_batched(c, {CopyDesc{Tt, b, T, b, b, b, 0.5, 0.5, 0}});
  svd_batched(c, {SVDDesc{T, b, b, b, sv.as<double>(), u.as<double>(), b, v.as<double>(), b}});
  std::vector<double> s(b);
  H2_HIP(hipMemcpyAsync(s.data(), sv.p, (size_t)b * sizeof(double), hipMemcpyDeviceToHost, c.s));
  H2_HIP(hipStreamSynchronize(c.s));
  for (double x : s) H2_CHECK(std::isfinite(x), H2_ENUMERIC, "global range finder: non-finite values");
  int k = 0;
  if (s[0] > 0)
    while (k < std::min(rank, b) && s[k] > EIG_CUT * s[0]) ++k;
  Bbuf.alloc((size_t)n * std::max(k, 1) * sizeof(double));
  if (k > 0) {
    std::vector<double> rs(k);
    for (int i = 0; i < k; ++i) rs[i] = std::sqrt(s[i]);
    DevBuf drs;
    upload(drs, rs);
    gemm_batched(c, {GemmDesc{q.as<double>(), u.as<double>(), Bbuf.as<double>(), n, k, b, n, b, n,
                              0, 0, 1.0, 0.0}});
    scale_columns(c, {ScaleDesc{Bbuf.as<double>(), n, n, k, drs.as<double>()}});
    H2_HIP(hipStreamSynchronize(c.s));
  }
  return k;
}

}  // namespace h2

using namespace h2;

extern "C" h2_status h2_build_lowrank(const h2_tree* tree, h2_sampler_fn sampler, void* ctx,
                                      const h2_opts* opts, int global_rank, hipStream_t stream,
                                      h2_matrix** out, h2_build_stats* stats) {
  bool conv = true;
  h2_status st = guarded_status([&] {
    H2_CHECK(tree && sampler && opts && out, H2_EINVAL, "null argument");
    H2_CHECK(global_rank >= 1, H2_EINVAL, "global rank must be >= 1");
    H2_CHECK(opts->tol > 0 && opts->tol < 1, H2_EINVAL, "tol must be in (0, 1)");
    H2_CHECK(opts->prec == H2_FP64, H2_EINVAL, "construction runs in FP64; convert afterwards");
    *out = nullptr;
    tree_device(tree);
    Ctx c;
    c.s = stream;
    UserSampler S(tree, sampler, ctx);
    BuildParams p;
    p.rank_cap = opts->rank_cap;
    p.oversample = opts->oversample;
    p.tol = opts->tol;
    p.adaptive = opts->adaptive != 0;
    p.max_rounds = opts->max_rounds;
    p.seed = opts->seed;
    p.iteration = 0;
    // ||H||_2 through the sampler, as a plain build estimates it
    double nu = opts->norm;
    int64_t norm_applies = 0;
    if (!(nu > 0)) {
      const int64_t a0 = S.applies;
      nu = power_norm_device(tree->n, [&](const double* v, double* w) { S.apply(c, 1, v, w); },
                             p.seed, 0, p.norm_rel, 3, 30, c.s, nullptr);
      norm_applies = S.applies - a0;
    }
    H2_CHECK(std::isfinite(nu) && nu > 0, H2_ENUMERIC, "norm estimate is zero or not finite");
    p.norm = nu;
    const int64_t a_global0 = S.applies;
    DevBuf B;
    const int k = global_lowrank(tree, S, global_rank, opts->oversample, p.seed, c, B);
    const int64_t a_global = S.applies - a_global0;
    // construction of the residual H - B B^T
    // (a global rank-k term adds up to k to every block's rank: the residual's
    // recompression gets that much more room)
    LowRankCorrected res(&S, B.as<double>(), tree->n, k, -1.0);
    h2_build_stats st_res{};
    bool conv_res = true;
    BuildParams pr = p;
    pr.dest_cap = p.rank_cap + k;
    auto Hres = build_h2(tree, res, pr, c, &st_res, &conv_res);
    // B B^T added back: recompress A_res + B B^T (no Hessian products)
    MatrixSampler ms(Hres.get());
    LowRankCorrected upd(&ms, B.as<double>(), tree->n, k, 1.0);
    BuildParams p2 = p;
    p2.iteration = 1;
    h2_build_stats st_upd{};
    bool conv_upd = true;
    auto H = build_h2(tree, upd, p2, c, &st_upd, &conv_upd);
    conv = conv_res && conv_upd;
    if (stats) {
      *stats = st_upd;
      for (int l = 0; l < H2_MAX_LEVELS; ++l) {
        stats->weak_rank[l] = st_res.weak_rank[l];
        stats->range_cols[l] = st_res.range_cols[l];
        stats->rounds[l] = st_res.rounds[l];
        stats->first_cols[l] = st_res.first_cols[l];
      }
      stats->applies = a_global + st_res.applies;
      stats->norm_applies = norm_applies;
      stats->norm = nu;
      stats->converged = conv ? 1 : 0;
      stats->global_rank = k;
      stats->global_applies = a_global;
      stats->update_applies = st_upd.applies;
    }
    *out = H.release();
  });
  if (st == H2_OK && !conv) return H2_ENOTCONVERGED;
  return st;
}
