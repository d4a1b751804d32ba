// Hierarchical Newton-Schulz inversion (Appendix A).  Alg. 1: the iteration
// X <- (2I - X A) X for a symmetric positive definite A started from a scaled
// identity; Alg. 2: every iterate is rebuilt by the construction of Sec. 3.3
// at a threshold eps_k chosen per iteration; Alg. 3: the sampler of the next
// iterate evaluates (2I - X_k A) X_k Omega, here as W = X_k Omega,
// Y = 2W - X_k (A W) -- three HGEMVs per block of samples.
//
// The residual E = ||I - A X||_2 is estimated by the power method on R^T R
// (R v = v - A (X v), R^T w = w - X (A w)); two significant digits by default
// (Sec. 3.2 norms).  Iterates are built to absolute accuracy eps_k / ||A||_2,
// the scale at which their error enters I - A X.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <functional>

#include "build.h"
#include "kernels_common.h"
#include "vecops.h"

namespace h2 {

h2_status guarded_status(const std::function<void()>& f);
void matrix_copy_convert(const h2_matrix* A, h2_matrix* B, double scale, hipStream_t s);
void matrix_identity(h2_matrix* A, const h2_tree* t, double alpha, hipStream_t s);

static double now_ms2() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Y = (2I - X A) X Omega in tree order
struct NSSampler : Sampler {
  const h2_matrix* X;
  const h2_matrix* A;
  DevBuf buf;
  NSSampler(const h2_matrix* x, const h2_matrix* a) : X(x), A(a) {}
  void apply(Ctx& c, int ncols, const double* om, double* y) override {
    if (ncols <= 0) return;
    const int n = X->tree->n;
    buf.reserve((size_t)2 * n * ncols * sizeof(double));
    double* W = buf.as<double>();
    double* T = W + (size_t)n * ncols;
    gemv_tree_f64(X, ncols, 1.0, om, n, 0.0, W, n, c.s);
    gemv_tree_f64(A, ncols, 1.0, W, n, 0.0, T, n, c.s);
    axpby(n, ncols, 2.0, W, n, 0.0, y, n, c.s);
    gemv_tree_f64(X, ncols, -1.0, T, n, 1.0, y, n, c.s);
    applies += ncols;
  }
};

__global__ void k_d2f(int n, int ncols, const double* __restrict__ a, int lda, float* __restrict__ b,
                      int ldb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * ncols) return;
  const int r = (int)(e % n), c = (int)(e / n);
  b[(size_t)c * ldb + r] = (float)a[(size_t)c * lda + r];
}

// y = 2 W - Z in FP64 from FP32 W, Z (n x ncols, ld n)
__global__ void k_two_w_minus(int n, int ncols, const float* __restrict__ w,
                              const float* __restrict__ z, double* __restrict__ y, int ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * ncols) return;
  const int r = (int)(e % n), c = (int)(e / n);
  y[(size_t)c * ldy + r] = 2.0 * (double)w[e] - (double)z[e];
}

// The same sampler with FP32 copies of X_k and A (FP32 HGEMVs on matrix
// cores); Omega arrives and Y leaves in FP64 for the FP64 construction.
struct NSSamplerF32 : Sampler {
  const h2_matrix* X;
  const h2_matrix* A;
  DevBuf buf;
  NSSamplerF32(const h2_matrix* x, const h2_matrix* a) : X(x), A(a) {}
  void apply(Ctx& c, int ncols, const double* om, double* y) override {
    if (ncols <= 0) return;
    const int n = X->tree->n;
    buf.reserve((size_t)4 * n * ncols * sizeof(float));
    float* O = buf.as<float>();
    float* W = O + (size_t)n * ncols;
    float* T = W + (size_t)n * ncols;
    float* Y = T + (size_t)n * ncols;
    const int64_t tot = (int64_t)n * ncols;
    const unsigned blocks = (unsigned)((tot + 255) / 256);
    k_d2f<<<blocks, 256, 0, c.s>>>(n, ncols, om, n, O, n);
    H2_LAUNCH_CHECK();
    gemv_tree_f32(X, ncols, 1.0f, O, n, 0.0f, W, n, c.s);
    gemv_tree_f32(A, ncols, 1.0f, W, n, 0.0f, T, n, c.s);
    gemv_tree_f32(X, ncols, 1.0f, T, n, 0.0f, Y, n, c.s);
    k_two_w_minus<<<blocks, 256, 0, c.s>>>(n, ncols, W, Y, y, n);
    H2_LAUNCH_CHECK();
    applies += ncols;
  }
};

// Samples of the order-l hyperpower iterate X_k (I + R + ... + R^(l-1)) Omega,
// R = I - A X_k, evaluated Horner-style (Appendix A.2, Alg. 4):
// Y = R = Omega; l - 1 times R <- R - A (X_k R), Y <- Y + R; then X_k Y.
struct HyperpowerSampler : Sampler {
  const h2_matrix* X;
  const h2_matrix* A;
  int order;
  DevBuf buf;
  HyperpowerSampler(const h2_matrix* x, const h2_matrix* a, int l) : X(x), A(a), order(l) {}
  void apply(Ctx& c, int ncols, const double* om, double* y) override {
    if (ncols <= 0) return;
    const int n = X->tree->n;
    const size_t blk = (size_t)n * ncols;
    buf.reserve(3 * blk * sizeof(double));
    double* R = buf.as<double>();
    double* Y = R + blk;
    double* T = Y + blk;
    axpby(n, ncols, 1.0, om, n, 0.0, R, n, c.s);
    axpby(n, ncols, 1.0, om, n, 0.0, Y, n, c.s);
    for (int i = 1; i < order; ++i) {
      gemv_tree_f64(X, ncols, 1.0, R, n, 0.0, T, n, c.s);
      gemv_tree_f64(A, ncols, -1.0, T, n, 1.0, R, n, c.s);
      axpby(n, ncols, 1.0, R, n, 1.0, Y, n, c.s);
    }
    gemv_tree_f64(X, ncols, 1.0, Y, n, 0.0, y, n, c.s);
    applies += ncols;
  }
};

// Sampler that applies one H2 matrix (tree order)
struct GemvSampler : Sampler {
  const h2_matrix* A;
  explicit GemvSampler(const h2_matrix* a) : A(a) {}
  void apply(Ctx& c, int ncols, const double* om, double* y) override {
    gemv_tree_f64(A, ncols, 1.0, om, A->tree->n, 0.0, y, A->tree->n, c.s);
    applies += ncols;
  }
};

// E = ||I - A X||_2 by the power method on R^T R (R v = v - A (X v),
// R^T w = w - X (A w)) for several (A, X) pairs in lock step
struct ResidJob {
  const h2_matrix* A;
  const h2_matrix* X;
  double rel;
  int max_it;
  uint64_t seed;
  uint32_t iteration;
  double E = 0;
  int iters = 0;
  std::vector<double> history;
};

void residual_norm_multi(std::vector<ResidJob>& rj, hipStream_t s, bool graph) {
  std::vector<DevBuf> tmp(rj.size());
  std::vector<PowerJob> pj(rj.size());
  for (size_t i = 0; i < rj.size(); ++i) {
    const h2_matrix* A = rj[i].A;
    const h2_matrix* X = rj[i].X;
    const int n = A->tree->n;
    tmp[i].alloc((size_t)2 * n * sizeof(double));
    double* t1 = tmp[i].as<double>();
    double* r = t1 + n;
    PowerJob& J = pj[i];
    J.n = n;
    J.op = [A, X, n, t1, r](const double* v, double* w, hipStream_t st) {
      // r = v - A (X v);  w = r - X (A r)
      gemv_tree_f64(X, 1, 1.0, v, n, 0.0, t1, n, st);
      H2_HIP(hipMemcpyAsync(r, v, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
      gemv_tree_f64(A, 1, -1.0, t1, n, 1.0, r, n, st);
      gemv_tree_f64(A, 1, 1.0, r, n, 0.0, t1, n, st);
      H2_HIP(hipMemcpyAsync(w, r, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
      gemv_tree_f64(X, 1, -1.0, t1, n, 1.0, w, n, st);
    };
    J.seed = rj[i].seed;
    J.iteration = rj[i].iteration;
    J.phase = PHASE_RESID;
    J.rel = rj[i].rel;
    J.min_it = 3;
    J.max_it = rj[i].max_it;
    J.sqrt_out = true;
  }
  power_norm_multi(pj, s, graph);
  for (size_t i = 0; i < rj.size(); ++i) {
    rj[i].E = pj[i].result;
    rj[i].iters = pj[i].iters;
    rj[i].history = std::move(pj[i].history);
  }
}

double residual_norm_device(const h2_matrix* A, const h2_matrix* X, double rel, int max_it,
                            uint64_t seed, uint32_t iteration, hipStream_t s) {
  std::vector<ResidJob> rj{{A, X, rel, max_it, seed, iteration}};
  residual_norm_multi(rj, s, false);
  return rj[0].E;
}

// Newton-Schulz for several independent matrices in lock step: every
// iteration evaluates each residual, then rebuilds all unfinished iterates in
// one batched construction (build_h2_multi).
struct NSJob {
  const h2_matrix* A = nullptr;
  h2_ns_opts o{};
  h2_ns_stats stats{};
  h2_status status = H2_ENOTCONVERGED;
  std::unique_ptr<h2_matrix> X;
  // state
  double nuA = 0, prevE = -1, eps_build = 0, norm_rel = 0, resid_rel = 0, switch_E = 0;
  bool low = false, active = true;
  BuildParams bp;
  std::unique_ptr<h2_matrix> A32, X32;
  std::unique_ptr<Sampler> S;
};

static std::unique_ptr<h2_matrix> to_f32(const h2_matrix* M, hipStream_t s) {
  auto B = std::make_unique<h2_matrix>();
  matrix_layout(B.get(), M->tree, M->rank);
  matrix_alloc(B.get(), H2_FP32);
  matrix_copy_convert(M, B.get(), 1.0, s);
  return B;
}

void ns_iterate_multi(std::vector<NSJob>& jobs, hipStream_t s) {
  const double t_begin = now_ms2();
  for (auto& J : jobs) {
    const h2_ns_opts& o = J.o;
    const h2_tree* t = J.A->tree;
    const int n = t->n;
    J.stats = h2_ns_stats{};
    J.status = H2_ENOTCONVERGED;
    J.active = true;
    J.prevE = -1;
    J.norm_rel = o.norm_rel > 0 ? o.norm_rel : 1e-2;
    J.resid_rel = o.resid_rel > 0 ? o.resid_rel : 1e-2;
    J.eps_build = o.eps_build > 0 ? o.eps_build : o.eps / 10.0;
    H2_CHECK(J.eps_build > 0, H2_EINVAL, "need eps > 0 or eps_build > 0");
    const h2_matrix* A = J.A;
    auto gop = [&](const double* v, double* w) { gemv_tree_f64(A, 1, 1.0, v, n, 0.0, w, n, s); };
    J.nuA = power_norm_device(n, gop, o.seed, 0, J.norm_rel, 3, J.norm_rel >= 1e-2 ? 30 : 500, s,
                              nullptr);
    H2_CHECK(std::isfinite(J.nuA) && J.nuA > 0, H2_ENUMERIC, "norm of A is zero or not finite");
    J.stats.norm = J.nuA;
    J.X = std::make_unique<h2_matrix>();
    if (o.x0 == 0) {
      matrix_identity(J.X.get(), t, 1.0 / J.nuA, s);
    } else if (o.x0 == 2) {
      matrix_layout(J.X.get(), t, o.x0_matrix->rank);
      matrix_alloc(J.X.get(), H2_FP64);
      matrix_copy_convert(o.x0_matrix, J.X.get(), 1.0, s);
    } else {
      matrix_layout(J.X.get(), t, A->rank);
      matrix_alloc(J.X.get(), H2_FP64);
      matrix_copy_convert(A, J.X.get(), 1.0 / (J.nuA * J.nuA), s);
    }
    J.bp = BuildParams{};
    J.bp.rank_cap = o.rank_cap > 0 ? o.rank_cap : t->leaf;
    J.bp.oversample = o.oversample;
    J.bp.adaptive = o.adaptive != 0;
    J.bp.max_rounds = o.max_rounds;
    J.bp.seed = o.seed;
    J.bp.norm = 1.0 / J.nuA;
    // mixed precision: FP32 copies of A and of each iterate feed the sampler
    // until E <= sqrt(eps) (or the iteration stops contracting), then FP64
    J.low = o.prec == H2_FP32;
    if (J.low) J.A32 = to_f32(A, s);
    J.switch_E = std::sqrt(std::max(o.eps, 0.0));
  }
  Ctx c;
  c.s = s;
  for (int k = 0;; ++k) {
    std::vector<BuildJob> bj;
    std::vector<NSJob*> who;
    // residuals of every unfinished problem in lock step, the power steps
    // replayed from a captured graph
    std::vector<ResidJob> rj;
    std::vector<NSJob*> rw;
    for (auto& J : jobs)
      if (J.active) {
        rj.push_back({J.A, J.X.get(), J.resid_rel, J.resid_rel >= 1e-2 ? 30 : 3000, J.o.seed,
                      (uint32_t)k});
        rw.push_back(&J);
      }
    {
      const double t0 = now_ms2();
      residual_norm_multi(rj, s, true);
      const double dt = now_ms2() - t0;
      for (NSJob* J : rw) J->stats.time_ms[0] += dt;
    }
    for (size_t q = 0; q < rw.size(); ++q) {
      NSJob& J = *rw[q];
      const h2_ns_opts& o = J.o;
      const double E = rj[q].E;
      H2_CHECK(std::isfinite(E), H2_ENUMERIC, "residual is not finite");
      if (k <= H2_MAX_NS_ITERS) J.stats.resid[k] = E;
      J.stats.iterations = k;
      if (o.eps > 0 && E <= o.eps) { J.status = H2_OK; J.active = false; continue; }
      if (k >= 1 && E > J.prevE && E > 1.0) { J.status = H2_EDIVERGED; J.active = false; continue; }
      if (k >= o.max_iter || k >= H2_MAX_NS_ITERS) { J.active = false; continue; }
      if (J.low && (E <= J.switch_E || (k >= 2 && E < 0.5 && E > 0.5 * J.prevE))) J.low = false;
      J.prevE = E;
      const double eps_k =
          o.dynamic ? std::min(std::max(0.1 * E * E, J.eps_build), 1e-2) : J.eps_build;
      J.bp.tol = eps_k;
      J.bp.iteration = (uint32_t)(k + 1);
      const int order = o.unroll > 0 ? (1 << o.unroll) : (o.order > 2 ? o.order : 2);
      if (J.low) {
        J.X32 = to_f32(J.X.get(), s);
        J.S = std::make_unique<NSSamplerF32>(J.X32.get(), J.A32.get());
        J.stats.low_iterations += 1;
      } else if (order > 2) {
        J.S = std::make_unique<HyperpowerSampler>(J.X.get(), J.A, order);
      } else {
        J.S = std::make_unique<NSSampler>(J.X.get(), J.A);
      }
      BuildJob b;
      b.t = J.A->tree;
      b.S = J.S.get();
      b.prm = J.bp;
      // FP32 samples carry rounding of about 1e-7 relative: the range basis
      // keeps only directions above it
      b.prm.rank_cut = J.low ? 1e-7 : 1e-13;
      bj.push_back(std::move(b));
      who.push_back(&J);
    }
    if (bj.empty()) break;
    const double t0 = now_ms2();
    build_h2_multi(bj, c);
    const double dt = now_ms2() - t0;
    for (size_t i = 0; i < bj.size(); ++i) {
      NSJob& J = *who[i];
      J.stats.time_ms[1] += dt;
      if (!J.low && J.o.prec == H2_FP32) J.stats.time_ms[2] += dt;
      J.stats.applies[k] = bj[i].stats.applies;
      int mr = 0;
      for (int l = 0; l <= J.A->tree->L; ++l) mr = std::max(mr, bj[i].stats.strong_rank[l]);
      J.stats.max_rank[k] = mr;
      J.X = std::move(bj[i].out);
      J.S.reset();
      if (verbose())
        std::fprintf(stderr, "[h2_ns] iteration %d (%s): E %.3e eps_k %.1e applies %lld max rank %d build %.1f ms (%zu problems)\n",
                     k, J.low ? "fp32" : "fp64", J.prevE, J.bp.tol, (long long)bj[i].stats.applies, mr, dt,
                     bj.size());
    }
  }
  for (auto& J : jobs) J.stats.time_ms[3] = now_ms2() - t_begin;
}

std::unique_ptr<h2_matrix> ns_iterate(const h2_matrix* A, const h2_ns_opts& o, hipStream_t s,
                                      h2_ns_stats* st, h2_status* status) {
  std::vector<NSJob> jobs(1);
  jobs[0].A = A;
  jobs[0].o = o;
  ns_iterate_multi(jobs, s);
  if (st) *st = jobs[0].stats;
  *status = jobs[0].status;
  return std::move(jobs[0].X);
}

}  // namespace h2

using namespace h2;

extern "C" {

void h2_ns_opts_default(h2_ns_opts* o) {
  if (!o) return;
  *o = h2_ns_opts{};
  o->eps = 1e-4;
  o->max_iter = 60;
  o->x0 = 0;
  o->dynamic = 1;
  o->eps_build = 0;
  o->norm_rel = 1e-2;
  o->resid_rel = 1e-2;
  o->rank_cap = 0;
  o->oversample = 10;
  o->adaptive = 1;
  o->max_rounds = 16;
  o->seed = 1;
  o->prec = H2_FP64;
  o->order = 0;
  o->unroll = 0;
  o->x0_matrix = nullptr;
}

// argument checks shared by the single and batched entry points
static void check_ns_opts(const h2_matrix* A, const h2_ns_opts& o) {
  H2_CHECK(o.max_iter >= 0, H2_EINVAL, "max_iter must be >= 0");
  H2_CHECK(o.prec == H2_FP64 || o.prec == H2_FP32, H2_EINVAL,
           "Newton-Schulz precision must be FP64 or FP32 (BF16 iterates cannot reach 1e-4)");
  H2_CHECK(o.x0 >= 0 && o.x0 <= 2, H2_EINVAL, "x0 must be 0, 1 or 2");
  H2_CHECK(o.order == 0 || (o.order >= 2 && o.order <= 1024), H2_EINVAL,
           "hyperpower order must be 0 or 2..1024");
  H2_CHECK(o.unroll >= 0 && o.unroll <= 10, H2_EINVAL, "unroll must be 0..10");
  H2_CHECK(o.unroll == 0 || o.order == 0, H2_EINVAL, "give either order or unroll");
  H2_CHECK(o.prec == H2_FP64 || (o.order <= 2 && o.unroll == 0), H2_EINVAL,
           "hyperpower and unrolled steps run in FP64");
  if (o.x0 == 2) {
    H2_CHECK(o.x0_matrix != nullptr, H2_EINVAL, "x0 = 2 needs x0_matrix");
    H2_CHECK(o.x0_matrix->tree == A->tree, H2_EINVAL, "x0_matrix must share A's tree");
    H2_CHECK(o.x0_matrix->st.prec == H2_FP64, H2_EINVAL, "x0_matrix must be FP64");
  }
}

h2_status h2_newton_schulz(const h2_matrix* A, const h2_ns_opts* opts, hipStream_t stream,
                           h2_matrix** X_out, h2_ns_stats* stats) {
  h2_status result = H2_OK;
  h2_status st = guarded_status([&] {
    H2_CHECK(A && opts && X_out, H2_EINVAL, "null argument");
    H2_CHECK(A->st.prec == H2_FP64, H2_EINVAL, "Newton-Schulz needs an FP64 matrix");
    check_ns_opts(A, *opts);
    auto X = ns_iterate(A, *opts, stream, stats, &result);
    *X_out = X.release();
  });
  return st != H2_OK ? st : result;
}

h2_status h2_newton_schulz_batched(int nprob, const h2_matrix* const* A, const h2_ns_opts* opts,
                                   hipStream_t stream, h2_matrix** X_out, h2_ns_stats* stats,
                                   h2_status* status) {
  return guarded_status([&] {
    H2_CHECK(nprob >= 0 && (nprob == 0 || (A && opts && X_out)), H2_EINVAL, "null argument");
    std::vector<NSJob> jobs(nprob);
    for (int i = 0; i < nprob; ++i) {
      X_out[i] = nullptr;
      H2_CHECK(A[i] && A[i]->st.prec == H2_FP64, H2_EINVAL, "Newton-Schulz needs FP64 matrices");
      check_ns_opts(A[i], opts[i]);
      jobs[i].A = A[i];
      jobs[i].o = opts[i];
    }
    ns_iterate_multi(jobs, stream);
    for (int i = 0; i < nprob; ++i) {
      if (stats) stats[i] = jobs[i].stats;
      if (status) status[i] = jobs[i].status;
      X_out[i] = jobs[i].X.release();
    }
  });
}

h2_status h2_residual_norm_batched(int nprob, const h2_matrix* const* A, const h2_matrix* const* X,
                                   double rel, int max_iter, uint64_t seed, uint32_t iteration,
                                   int graph, hipStream_t stream, double* out, int* iters,
                                   double* history) {
  return guarded_status([&] {
    H2_CHECK(nprob >= 0 && (nprob == 0 || (A && X && out)), H2_EINVAL, "null argument");
    std::vector<ResidJob> rj;
    const int mi = max_iter > 0 ? max_iter : 30;
    for (int i = 0; i < nprob; ++i) {
      H2_CHECK(A[i] && X[i] && A[i]->tree == X[i]->tree, H2_EINVAL, "A and X must share a tree");
      H2_CHECK(A[i]->st.prec == H2_FP64 && X[i]->st.prec == H2_FP64, H2_EINVAL,
               "FP64 matrices needed");
      rj.push_back({A[i], X[i], rel > 0 ? rel : 1e-2, mi, seed, iteration});
    }
    residual_norm_multi(rj, stream, graph != 0);
    for (int i = 0; i < nprob; ++i) {
      out[i] = rj[i].E;
      if (iters) iters[i] = rj[i].iters;
      if (history)
        for (int q = 0; q < mi; ++q)
          history[(size_t)i * mi + q] = q < (int)rj[i].history.size() ? rj[i].history[q] : 0.0;
    }
  });
}

h2_status h2_residual_norm(const h2_matrix* A, const h2_matrix* X, double rel, int max_iter,
                           uint64_t seed, uint32_t iteration, hipStream_t stream, double* out) {
  return guarded_status([&] {
    H2_CHECK(A && X && out, H2_EINVAL, "null argument");
    H2_CHECK(A->tree == X->tree, H2_EINVAL, "A and X must share a tree");
    H2_CHECK(A->st.prec == H2_FP64 && X->st.prec == H2_FP64, H2_EINVAL, "FP64 matrices needed");
    *out = residual_norm_device(A, X, rel > 0 ? rel : 1e-2, max_iter > 0 ? max_iter : 30, seed,
                                iteration, stream);
  });
}

int h2_sampler_h2_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega, double* y,
                        int ld_y, hipStream_t stream) {
  h2_status st = h2_gemv((const h2_matrix*)ctx, ncols, 1.0, omega, ld_omega, 0.0, y, ld_y, stream);
  (void)n;
  return st == H2_OK ? 0 : 1;
}

}  // extern "C"
