// Construction of an H2 approximation from products with blocks of vectors
// (Sec. 3.3), followed by recompression into the strong partition (Sec. 3.2).
//
// Peeling on the weak (sibling) partition, coarse to fine.  At level l the
// sampling matrix is Gaussian on the rows of every left child t1 = 2p and zero
// elsewhere, so Y[t2] samples the block A[t2, t1] of every sibling pair at
// once after the coarser levels' low-rank blocks are removed.  Rounds repeat
// until the Halko-Martinsson-Tropp estimate of every pair is below tau; a QR of
// the samples with a numerical-rank SVD cut gives the range basis Q0, the
// product A [0; Q0] gives B0 = A[t1, t2] Q0, and a truncated SVD of B0 gives
// the factors Q (on t2) and B (on t1) with A[t2, t1] ~ Q B^T.
//
// Recompression (QR downsweep of block rows, truncated-SVD upsweep, projection)
// folds the weak factors into nested bases U / E, couplings S and dense near
// blocks D of the strong partition of the tree.
//
// Thresholds: tau = eps * nu / (4 L) for the sampled blocks and the bases;
// numerical-rank cut 1e-13 sigma_1 for the range basis, whose columns take a
// canonical sign (largest-magnitude entry positive) because one projection
// matrix carries the bases of all pairs of a level and a tau-sized residual of
// the coarser levels couples neighbouring pairs.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <functional>
#include <map>
#include <tuple>

#include "build.h"
#include "mlp.h"
#include "kernels_common.h"
#include "vecops.h"

namespace h2 {

constexpr int TSQR_MIN_ROWS = 96;

void keep_factors(int l, const std::vector<int>& k, int K, const double* F_dev, int n);
void reset_factors();

static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ samplers
void UserSampler::apply(Ctx& c, int ncols, const double* om, double* y) {
  if (ncols <= 0) return;
  const int n = t->n;
  buf.reserve((size_t)2 * n * ncols * sizeof(double));
  double* om_u = buf.as<double>();
  double* y_u = om_u + (size_t)n * ncols;
  scatter_rows(t, ncols, 1.0, om, n, 0.0, om_u, n, c.s);
  const int rc = fn(ctx, n, ncols, om_u, n, y_u, n, c.s);
  if (rc != 0) throw Error(H2_ECALLBACK, "sampler callback returned " + std::to_string(rc));
  H2_HIP(hipGetLastError());
  gather_rows(t, ncols, y_u, n, y, n, c.s);
  applies += ncols;
}

// ------------------------------------------------------------------ kernels
// Omega of level l: Gaussian on the rows of even (left) clusters, zero elsewhere
__global__ void k_fill_left(uint64_t key, int n, int ncols, int nclus,
                            const int32_t* __restrict__ start, double* __restrict__ om) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * ncols) return;
  const int r = (int)(e % n), j = (int)(e / n);
  int lo = 0, hi = nclus - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= r) lo = mid; else hi = mid - 1;
  }
  om[(size_t)j * n + r] = (lo & 1) ? 0.0 : gauss_entry(key, (uint64_t)r, (uint64_t)j);
}

// stacked identities on the leaves: column q of leaf t has a 1 in its q-th row
__global__ void k_fill_diag(int n, int ncols, int nleaf, const int32_t* __restrict__ start,
                            double* __restrict__ om) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * ncols) return;
  const int r = (int)(e % n), j = (int)(e / n);
  int lo = 0, hi = nleaf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= r) lo = mid; else hi = mid - 1;
  }
  om[(size_t)j * n + r] = (r - start[lo] == j) ? 1.0 : 0.0;
}

// D = (M + M^T) / 2 of the leading m x m block of M (column-major, ld)
struct SymDesc {
  const double* M;
  int ld, m;
  double* D;
};
__global__ void k_sym(const SymDesc* __restrict__ ds) {
  const SymDesc d = ds[blockIdx.x];
  for (int e = threadIdx.x; e < d.m * d.m; e += blockDim.x) {
    const int i = e % d.m, j = e / d.m;
    d.D[(size_t)j * d.m + i] = 0.5 * (d.M[(size_t)j * d.ld + i] + d.M[(size_t)i * d.ld + j]);
  }
}

__global__ void k_nonfinite(int64_t n, const double* __restrict__ v, int* flag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && !isfinite(v[e])) *flag = 1;
}

// ------------------------------------------------------------------ helpers
namespace {

struct Pair {
  int a1, m1, a2, m2;  // t1 rows [a1, a1+m1), t2 rows [a2, a2+m2)
};

struct Level {
  int K = 0;               // max pair rank
  std::vector<int> k;      // pair ranks
  DevBuf F;                // n x K, column-major: B on t1 rows, Q on t2 rows
};

template <class T>
std::vector<T> to_host(const T* d, size_t n, hipStream_t s) {
  std::vector<T> h(n);
  if (n) {
    H2_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    H2_HIP(hipStreamSynchronize(s));
  }
  return h;
}

void check_finite(Ctx& c, const double* v, int64_t n, const char* what) {
  if (n <= 0) return;
  DevBuf flag(sizeof(int));
  H2_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), c.s));
  k_nonfinite<<<(unsigned)((n + 255) / 256), 256, 0, c.s>>>(n, v, flag.as<int>());
  H2_LAUNCH_CHECK();
  int h = 0;
  H2_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, c.s));
  H2_HIP(hipStreamSynchronize(c.s));
  H2_CHECK(h == 0, H2_ENUMERIC, std::string("non-finite values in ") + what);
}

// Y -= sum_{l' < lmax} Atilde_{l'} Om (n x ncols, ld n)
void subtract_levels(Ctx& c, const h2_tree* t, const std::vector<Level>& lv, int lmax,
                     const double* om, double* y, int ncols) {
  const int n = t->n;
  for (int l = 1; l < lmax; ++l) {
    const Level& L = lv[l];
    if (L.K == 0) continue;
    const double* F = L.F.as<double>();
    std::vector<GemmDesc> red, upd;
    const int np = 1 << (l - 1);
    std::vector<double*> c1(np), c2(np);
    for (int p = 0; p < np; ++p) {
      const int k = L.k[p];
      if (k == 0) continue;
      const int a1 = t->cstart[cid(l, 2 * p)], m1 = t->csize[cid(l, 2 * p)];
      const int a2 = t->cstart[cid(l, 2 * p + 1)], m2 = t->csize[cid(l, 2 * p + 1)];
      c1[p] = c.scratch.get((size_t)k * ncols);
      c2[p] = c.scratch.get((size_t)k * ncols);
      red.push_back({F + a1, om + a1, c1[p], k, ncols, m1, n, n, k, 1, 0, 1.0, 0.0});
      red.push_back({F + a2, om + a2, c2[p], k, ncols, m2, n, n, k, 1, 0, 1.0, 0.0});
      upd.push_back({F + a2, c1[p], y + a2, m2, ncols, k, n, k, n, 0, 0, -1.0, 1.0});
      upd.push_back({F + a1, c2[p], y + a1, m1, ncols, k, n, k, n, 0, 0, -1.0, 1.0});
    }
    gemm_batched(c, red);
    gemm_batched(c, upd);
  }
}

// Left singular vectors and singular values of X (M x K, column-major, ld):
// K >= M: Jacobi on X^T; K < M: QR then Jacobi on R^T.  Writes U (M x r,
// ld M) with r = min(M, K) and sigma (r).  X is destroyed.
struct LsvTask {
  double* X;
  int ld, M, K;
  double* U;      // M x min(M,K)
  double* sigma;  // min(M,K)
};

void left_svd_batched(Ctx& c, const std::vector<LsvTask>& tasks) {
  std::vector<CopyDesc> tr;
  std::vector<QRDesc> qrs;
  std::vector<SVDDesc> svs;
  std::vector<GemmDesc> back;
  for (const auto& tk : tasks) {
    if (tk.M == 0 || tk.K == 0) continue;
    if (tk.K >= tk.M) {
      double* Xt = c.scratch.get((size_t)tk.K * tk.M);
      tr.push_back({tk.X, tk.ld, Xt, tk.K, tk.K, tk.M, 1.0, 0.0, 1});
      svs.push_back({Xt, tk.K, tk.K, tk.M, tk.sigma, nullptr, 0, tk.U, tk.M});
    } else {
      double* Q = c.scratch.get((size_t)tk.M * tk.K);
      double* R = c.scratch.get((size_t)tk.K * tk.K);
      double* Rt = c.scratch.get((size_t)tk.K * tk.K);
      double* V = c.scratch.get((size_t)tk.K * tk.K);
      qrs.push_back({tk.X, tk.ld, tk.M, tk.K, Q, tk.M, R, tk.K});
      tr.push_back({R, tk.K, Rt, tk.K, tk.K, tk.K, 1.0, 0.0, 1});
      svs.push_back({Rt, tk.K, tk.K, tk.K, tk.sigma, nullptr, 0, V, tk.K});
      back.push_back({Q, V, tk.U, tk.M, tk.K, tk.K, tk.M, tk.K, tk.M, 0, 0, 1.0, 0.0});
    }
  }
  qr_auto(c, qrs);
  copy_batched(c, tr);
  svd_batched(c, svs);
  gemm_batched(c, back);
}

}  // namespace

// Features of the sibling pairs of level l for the rank predictor (the list
// is documented with h2_mlp_create): geometry of t2, tolerance, and the
// singular-value decay and rank of the parent pair.
std::vector<float> pair_features(const h2_tree* t, int l, double tol,
                                 const std::vector<std::vector<double>>& psig,
                                 const std::vector<int>& pk) {
  const int np = 1 << (l - 1), D = t->dim;
  double root = 0;
  for (int d = 0; d < D; ++d) root = std::max(root, t->hi[0][d] - t->lo[0][d]);
  if (!(root > 0)) root = 1.0;
  static const int sidx[7] = {2, 4, 8, 16, 32, 64, 128};
  std::vector<float> f((size_t)np * H2_MLP_FEATURES, 0.0f);
  for (int p = 0; p < np; ++p) {
    float* fp = f.data() + (size_t)p * H2_MLP_FEATURES;
    const int c2 = 2 * p + 1;
    std::vector<double> ext(D);
    for (int d = 0; d < D; ++d) ext[d] = t->hi[l][(size_t)c2 * D + d] - t->lo[l][(size_t)c2 * D + d];
    std::sort(ext.begin(), ext.end(), std::greater<double>());
    fp[0] = (float)((double)l / t->L);
    fp[1] = (float)(std::log2((double)t->csize[cid(l, c2)]) / 16.0);
    for (int d = 0; d < std::min(D, 3); ++d) fp[2 + d] = (float)(ext[d] / root);
    const double dd = 1e-12 * root;
    fp[5] = D > 1 ? (float)(std::log10((ext[0] + dd) / (ext[D - 1] + dd)) / 4.0) : 0.0f;
    fp[6] = (float)(D / 3.0);
    fp[7] = (float)(std::log10(tol) / 10.0);
    if (l == 1) {
      fp[15] = -1.0f;
      continue;
    }
    const std::vector<double>& s = psig[p / 2];
    for (int q = 0; q < 7; ++q) {
      const int i = sidx[q];
      double v = -1.0;
      if ((int)s.size() >= i && s[0] > 0) {
        const double r = s[i - 1] / s[0];
        v = r > 0 ? std::max(std::log10(r), -16.0) / 16.0 : -1.0;
      }
      fp[8 + q] = (float)v;
    }
    fp[15] = (float)(std::log2(1.0 + pk[p / 2]) / 10.0);
  }
  return f;
}

// ------------------------------------------------------------------ driver
std::unique_ptr<h2_matrix> build_h2(const h2_tree* t, Sampler& S, const BuildParams& prm, Ctx& c,
                                    h2_build_stats* st, bool* converged_out) {
  tree_device(t);
  const int n = t->n, L = t->L;
  const int b = prm.rank_cap + prm.oversample;
  H2_CHECK(b >= 1 && prm.rank_cap >= 1, H2_EINVAL, "rank_cap + oversample must be >= 1");
  H2_CHECK(!prm.adaptive || prm.max_rounds >= 2, H2_EINVAL, "adaptive mode needs max_rounds >= 2");
  H2_CHECK(b <= (prm.adaptive ? 512 : 1024), H2_EINVAL,
           "rank_cap + oversample must be <= 512 (adaptive) or 1024 (one round)");
  // the per-pair sample store holds at most 1024 columns (QR / SVD limit):
  // the round budget is clamped to what fits
  h2_build_stats local{};
  h2_build_stats& stats = st ? *st : local;
  stats = h2_build_stats{};
  stats.levels = L;
  const double t_start = now_ms();
  const int64_t applies0 = S.applies;
  bool converged = true;

  // ---- norm estimate (power method through the sampler)
  double t0 = now_ms();
  double nu = prm.norm;
  if (!(nu > 0)) {
    nu = power_norm_device(n, [&](const double* v, double* w) { S.apply(c, 1, v, w); }, prm.seed,
                           prm.iteration, prm.norm_rel, 3, prm.norm_rel >= 1e-2 ? 30 : 500, c.s,
                           nullptr);
  }
  H2_CHECK(std::isfinite(nu), H2_ENUMERIC, "norm estimate is not finite");
  stats.norm = nu;
  stats.norm_applies = S.applies - applies0;
  const int64_t applies1 = S.applies;
  stats.time_ms[0] = now_ms() - t0;
  const double tau = prm.tol * nu / (4.0 * std::max(L, 1));
  const double kHMT = 10.0 * std::sqrt(2.0 / M_PI);

  std::vector<Level> lv(L + 1);
  std::vector<std::vector<double>> prev_sig;   // singular values of B0 per pair, previous level
  std::vector<int> prev_k;
  DevBuf om_buf, y_buf;
  reset_factors();
  for (int l = 1; l <= L; ++l) {
    const int np = 1 << (l - 1);
    std::vector<Pair> pr(np);
    for (int p = 0; p < np; ++p)
      pr[p] = {t->cstart[cid(l, 2 * p)], t->csize[cid(l, 2 * p)], t->cstart[cid(l, 2 * p + 1)],
               t->csize[cid(l, 2 * p + 1)]};
    // first-round width: learned prediction (adaptive mode) or the plain width
    int b0 = b;
    std::vector<float> feats;
    if (prm.adaptive && (prm.mlp || records_on())) feats = pair_features(t, l, prm.tol, prev_sig, prev_k);
    if (prm.adaptive && prm.mlp) {
      auto* dX = (float*)c.stage.put(feats.data(), feats.size() * sizeof(float), c.s);
      DevBuf dy((size_t)np * sizeof(float));
      mlp_forward(prm.mlp, np, dX, dy.as<float>(), c.s);
      std::vector<float> pred(np);
      H2_HIP(hipMemcpyAsync(pred.data(), dy.p, np * sizeof(float), hipMemcpyDeviceToHost, c.s));
      H2_HIP(hipStreamSynchronize(c.s));
      c.stage.reset();
      float ymax = -1e30f;
      for (float v : pred) {
        H2_CHECK(std::isfinite(v), H2_ENUMERIC, "non-finite rank prediction");
        ymax = std::max(ymax, v);
      }
      const double kpred = std::max(0.0, std::expm1((double)ymax));
      b0 = (int)std::min<double>(std::max<double>(b, std::ceil(kpred) + prm.oversample), 1024 - b);
      b0 = std::max(b0, b);
    }
    stats.first_cols[l] = b0;
    const int max_rounds = std::max(2, std::min(prm.max_rounds, 1 + (1024 - b0) / b));
    const int cmax = prm.adaptive ? b0 + (max_rounds - 1) * b : b;
    // per-pair sample storage Z_p (m2 x cmax, ld m2) and an orthonormal basis
    // Qe_p of the samples kept so far (block Gram-Schmidt with two projections
    // per round), used by the estimator and by the final range basis
    std::vector<int64_t> zoff(np + 1, 0), qoff(np + 1, 0);
    for (int p = 0; p < np; ++p) {
      zoff[p + 1] = zoff[p] + (int64_t)pr[p].m2 * cmax;
      qoff[p + 1] = qoff[p] + (int64_t)pr[p].m2 * std::min(pr[p].m2, cmax);
    }
    DevBuf zbuf(std::max<int64_t>(zoff[np], 1) * sizeof(double));
    DevBuf qbuf(std::max<int64_t>(qoff[np], 1) * sizeof(double));
    double* Z = zbuf.as<double>();
    double* Qe = qbuf.as<double>();
    std::vector<int> cols(np, 0), qc(np, 0), needed(np, -1);
    std::vector<char> frozen(np, 0);
    om_buf.reserve((size_t)n * b0 * sizeof(double));
    y_buf.reserve((size_t)n * b0 * sizeof(double));
    double* om = om_buf.as<double>();
    double* y = y_buf.as<double>();
    int r = 0;
    DevBuf ebuf(np * sizeof(double));
    t0 = now_ms();
    while (true) {
      const int bw = r == 0 ? b0 : b;   // the first round may be wider (learned counts)
      const uint64_t key = stream_key(prm.seed, PHASE_RANGE, l, r, prm.iteration);
      const int64_t tot = (int64_t)n * bw;
      k_fill_left<<<(unsigned)((tot + 255) / 256), 256, 0, c.s>>>(
          key, n, bw, 1 << l, t->d_cstart.as<int32_t>() + cid(l, 0), om);
      H2_LAUNCH_CHECK();
      S.apply(c, bw, om, y);
      subtract_levels(c, t, lv, l, om, y, bw);
      if (r == 0) check_finite(c, y, (int64_t)n * bw, "samples");
      std::vector<int> newly(np, 0);
      std::vector<int> act;                    // pairs that take this round's samples
      for (int p = 0; p < np; ++p)
        if (!frozen[p]) act.push_back(p);
      // projected samples Yp'' = (I - Qe Qe^T)^2 Y[t2] (round 0: the samples)
      std::vector<double*> Yproj(np, nullptr);
      {
        std::vector<CopyDesc> cp;
        std::vector<GemmDesc> g1, g2, g3, g4;
        for (int p : act) {
          const int m2 = pr[p].m2;
          Yproj[p] = c.scratch.get((size_t)m2 * bw);
          cp.push_back({y + pr[p].a2, n, Yproj[p], m2, m2, bw, 1.0, 0.0, 0});
          const int q = qc[p];
          if (q == 0) continue;
          double* W1 = c.scratch.get((size_t)q * bw);
          double* W2 = c.scratch.get((size_t)q * bw);
          double* Qp_ = Qe + qoff[p];
          g1.push_back({Qp_, Yproj[p], W1, q, bw, m2, m2, m2, q, 1, 0, 1.0, 0.0});
          g2.push_back({Qp_, W1, Yproj[p], m2, bw, q, m2, q, m2, 0, 0, -1.0, 1.0});
          g3.push_back({Qp_, Yproj[p], W2, q, bw, m2, m2, m2, q, 1, 0, 1.0, 0.0});
          g4.push_back({Qp_, W2, Yproj[p], m2, bw, q, m2, q, m2, 0, 0, -1.0, 1.0});
        }
        copy_batched(c, cp);
        gemm_batched(c, g1);
        gemm_batched(c, g2);
        gemm_batched(c, g3);
        gemm_batched(c, g4);
      }
      if (prm.adaptive && r >= 1) {
        std::vector<CopyDesc> res_blocks;
        for (int p : act) res_blocks.push_back({Yproj[p], pr[p].m2, nullptr, 0, pr[p].m2, bw, 1.0, 0.0, 0});
        colnorm_max_batched(c, res_blocks, ebuf.as<double>());
        auto e = to_host(ebuf.as<double>(), res_blocks.size(), c.s);
        for (size_t q = 0; q < act.size(); ++q) {
          H2_CHECK(std::isfinite(e[q]), H2_ENUMERIC, "non-finite samples");
          if (kHMT * e[q] <= tau) {
            newly[act[q]] = 1;
            needed[act[q]] = cols[act[q]];   // columns that sufficed, before this probe round
          }
        }
      }
      // append this round's samples
      std::vector<CopyDesc> app;
      for (int p : act) {
        app.push_back({y + pr[p].a2, n, Z + zoff[p] + (size_t)cols[p] * pr[p].m2, pr[p].m2,
                       pr[p].m2, bw, 1.0, 0.0, 0});
        cols[p] += bw;
      }
      copy_batched(c, app);
      // extend Qe with the projected block: QR, one more projection, QR again
      // (tall panels by TSQR over many workgroups, short ones in one workgroup)
      {
        std::vector<QRDesc> q1, q2, t1, t2;
        std::vector<GemmDesc> g1, g2;
        std::vector<CopyDesc> put;
        for (int p : act) {
          const int m2 = pr[p].m2, q = qc[p];
          if (q >= m2) continue;
          const int kn = std::min(m2, bw);
          const int take = std::min(kn, m2 - q);
          const bool tall = m2 >= 2 * TSQR_MIN_ROWS && bw <= 96;  // else shape dispatch
          double* Qn = c.scratch.get((size_t)m2 * kn);
          double* Qn2 = c.scratch.get((size_t)m2 * kn);
          (tall ? t1 : q1).push_back({Yproj[p], m2, m2, bw, Qn, m2, nullptr, 0});
          if (q > 0) {
            double* Wq = c.scratch.get((size_t)q * kn);
            g1.push_back({Qe + qoff[p], Qn, Wq, q, kn, m2, m2, m2, q, 1, 0, 1.0, 0.0});
            g2.push_back({Qe + qoff[p], Wq, Qn, m2, kn, q, m2, q, m2, 0, 0, -1.0, 1.0});
            (tall ? t2 : q2).push_back({Qn, m2, m2, kn, Qn2, m2, nullptr, 0});
            put.push_back({Qn2, m2, Qe + qoff[p] + (size_t)q * m2, m2, m2, take, 1.0, 0.0, 0});
          } else {
            put.push_back({Qn, m2, Qe + qoff[p], m2, m2, take, 1.0, 0.0, 0});
          }
          qc[p] = q + take;
        }
        qr_auto(c, q1);
        qr_tall_batched(c, t1);
        gemm_batched(c, g1);
        gemm_batched(c, g2);
        qr_auto(c, q2);
        qr_tall_batched(c, t2);
        copy_batched(c, put);
      }
      for (int p = 0; p < np; ++p)
        if (newly[p]) frozen[p] = 1;
      ++r;
      H2_HIP(hipStreamSynchronize(c.s));
      c.scratch.clear();
      c.stage.reset();
      if (!prm.adaptive) break;
      bool all = true;
      for (int p = 0; p < np; ++p) all = all && frozen[p];
      if (r >= 2 && all) break;
      if (r >= max_rounds) { converged = false; break; }
    }
    stats.rounds[l] = r;
    stats.time_ms[1] += now_ms() - t0;

    // ---- range basis: Z = Qe (Qe^T Z); SVD of Qe^T Z, singular values above
    // 1e-13 sigma_1 (the left singular vectors of the samples)
    t0 = now_ms();
    std::vector<int> kq(np), k0(np, 0);
    std::vector<double*> Vp(np), sig(np);
    std::vector<int64_t> soff(np + 1, 0);
    for (int p = 0; p < np; ++p) soff[p + 1] = soff[p] + qc[p];
    double* sig_all = c.scratch.get(std::max<int64_t>(soff[np], 1));
    {
      std::vector<GemmDesc> g;
      std::vector<SVDDesc> svs;
      for (int p = 0; p < np; ++p) {
        const int m2 = pr[p].m2, cp = cols[p];
        kq[p] = qc[p];
        // Rt = Z^T Qe (cp x kq) = (Qe^T Z)^T
        double* Rt = c.scratch.get((size_t)cp * kq[p]);
        Vp[p] = c.scratch.get((size_t)kq[p] * kq[p]);
        sig[p] = sig_all + soff[p];
        g.push_back({Z + zoff[p], Qe + qoff[p], Rt, cp, kq[p], m2, m2, m2, cp, 1, 0, 1.0, 0.0});
        // left singular vectors of R = right singular vectors of R^T
        svs.push_back({Rt, cp, cp, kq[p], sig[p], nullptr, 0, Vp[p], kq[p]});
      }
      gemm_batched(c, g);
      svd_batched(c, svs);
    }
    std::vector<double*> Q0(np);
    int K0 = 0;
    {
      std::vector<GemmDesc> g;
      auto sh = to_host(sig_all, soff[np], c.s);
      for (int p = 0; p < np; ++p) {
        const double* s = sh.data() + soff[p];
        int k = 0;
        if (kq[p] > 0 && s[0] > 0) {
          H2_CHECK(std::isfinite(s[0]), H2_ENUMERIC, "non-finite singular values");
          while (k < kq[p] && s[k] > 1e-13 * s[0]) ++k;
        }
        k0[p] = k;
        K0 = std::max(K0, k);
        Q0[p] = c.scratch.get((size_t)pr[p].m2 * std::max(k, 1));
        if (k > 0) g.push_back({Qe + qoff[p], Vp[p], Q0[p], pr[p].m2, k, kq[p], pr[p].m2, kq[p], pr[p].m2, 0, 0, 1.0, 0.0});
      }
      gemm_batched(c, g);
      // canonical column signs: the projection below carries every pair's
      // basis in the same columns, so the result must not depend on signs
      std::vector<CopyDesc> cs;
      for (int p = 0; p < np; ++p)
        if (k0[p] > 0) cs.push_back({Q0[p], pr[p].m2, nullptr, 0, pr[p].m2, k0[p], 1.0, 0.0, 0});
      canonical_signs(c, cs);
    }
    stats.range_cols[l] = K0;
    H2_HIP(hipStreamSynchronize(c.s));
    zbuf.release();
    qbuf.release();
    stats.time_ms[2] += now_ms() - t0;

    // ---- projection B0 = (A [0; Q0])[t1] and truncation
    t0 = now_ms();
    Level& LV = lv[l];
    LV.k.assign(np, 0);
    std::vector<std::vector<double>> cur_sig(np);
    if (K0 > 0) {
      om_buf.reserve((size_t)n * K0 * sizeof(double));
      y_buf.reserve((size_t)n * K0 * sizeof(double));
      om = om_buf.as<double>();
      y = y_buf.as<double>();
      zero_block(c, om, n, K0, n);
      std::vector<CopyDesc> put;
      for (int p = 0; p < np; ++p)
        if (k0[p] > 0) put.push_back({Q0[p], pr[p].m2, om + pr[p].a2, n, pr[p].m2, k0[p], 1.0, 0.0, 0});
      copy_batched(c, put);
      S.apply(c, K0, om, y);
      subtract_levels(c, t, lv, l, om, y, K0);
      // truncated SVD of B0 (m1 x k0) by one-sided Jacobi:
      //   mode 0 (m1 >= k0, small k0): B0 V = U S         -> Q = Q0 V_k, B = U_k S_k
      //   mode 1 (m1 <  k0):  B0^T V = U S, B0 = V S U^T  -> Q = Q0 U_k, B = V_k S_k
      //   mode 2 (m1 >= k0, large k0): B0 = Q_B R (blocked QR), R^T V = U S,
      //          B0 = (Q_B V) S U^T                        -> Q = Q0 U_k, B = Q_B V_k S_k
      std::vector<CopyDesc> b0c, rtc;
      std::vector<CholQRDesc> bqr;
      std::vector<SVDDesc> svs;
      std::vector<int> kb(np, 0), mode(np, 0);
      std::vector<double*> Ub(np), Vb(np), sb(np), QB(np, nullptr);
      std::vector<int64_t> boff(np + 1, 0);
      for (int p = 0; p < np; ++p) boff[p + 1] = boff[p] + std::min(pr[p].m1, k0[p]);
      double* sb_all = c.scratch.get(std::max<int64_t>(boff[np], 1));
      for (int p = 0; p < np; ++p) {
        if (k0[p] == 0) continue;
        const int m1 = pr[p].m1, kk = k0[p];
        kb[p] = std::min(m1, kk);
        sb[p] = sb_all + boff[p];
        if (m1 >= kk && kk >= 96 && m1 >= 128) {
          mode[p] = 2;
          QB[p] = c.scratch.get((size_t)m1 * kk);
          double* RB = c.scratch.get((size_t)kk * kk);
          double* RBt = c.scratch.get((size_t)kk * kk);
          b0c.push_back({y + pr[p].a1, n, QB[p], m1, m1, kk, 1.0, 0.0, 0});
          bqr.push_back({QB[p], m1, m1, kk, RB, kk});
          rtc.push_back({RB, kk, RBt, kk, kk, kk, 1.0, 0.0, 1});
          Ub[p] = c.scratch.get((size_t)kk * kk);
          Vb[p] = c.scratch.get((size_t)kk * kk);
          svs.push_back({RBt, kk, kk, kk, sb[p], Ub[p], kk, Vb[p], kk});
          continue;
        }
        const bool tall = m1 >= kk;
        mode[p] = tall ? 0 : 1;
        const int mm = tall ? m1 : kk, nn = tall ? kk : m1;
        double* X = c.scratch.get((size_t)mm * nn);
        // a transposed copy reads B0 (m1 x k0 at y + a1, ld n) as its source
        b0c.push_back({y + pr[p].a1, n, X, mm, mm, nn, 1.0, 0.0, tall ? 0 : 1});
        Ub[p] = c.scratch.get((size_t)mm * nn);
        Vb[p] = c.scratch.get((size_t)nn * nn);
        svs.push_back({X, mm, mm, nn, sb[p], Ub[p], mm, Vb[p], nn});
      }
      copy_batched(c, b0c);
      qr_blocked(c, bqr);
      copy_batched(c, rtc);
      svd_batched(c, svs);
      auto sbh = to_host(sb_all, boff[np], c.s);
      for (int p = 0; p < np; ++p) cur_sig[p].assign(sbh.data() + boff[p], sbh.data() + boff[p] + kb[p]);
      for (int p = 0; p < np; ++p) {
        if (k0[p] == 0) continue;
        const double* s = sbh.data() + boff[p];
        int k = 0;
        while (k < kb[p] && s[k] > tau) ++k;
        H2_CHECK(kb[p] == 0 || std::isfinite(s[0]), H2_ENUMERIC, "non-finite singular values");
        LV.k[p] = k;
      }
      LV.K = *std::max_element(LV.k.begin(), LV.k.end());
      LV.F.alloc((size_t)n * std::max(LV.K, 1) * sizeof(double));
      double* F = LV.F.as<double>();
      zero_block(c, F, n, std::max(LV.K, 1), n);
      std::vector<GemmDesc> g;
      std::vector<CopyDesc> cb;
      std::vector<ScaleDesc> sc;
      for (int p = 0; p < np; ++p) {
        const int k = LV.k[p];
        if (k == 0) continue;
        const int m1 = pr[p].m1, m2 = pr[p].m2, kk = k0[p];
        if (mode[p] == 2) {
          g.push_back({Q0[p], Ub[p], F + pr[p].a2, m2, k, kk, m2, kk, n, 0, 0, 1.0, 0.0});
          g.push_back({QB[p], Vb[p], F + pr[p].a1, m1, k, kk, m1, kk, n, 0, 0, 1.0, 0.0});
        } else {
          const bool tall = mode[p] == 0;
          // right singular vectors of B0 (k0 x kb) and left ones (m1 x kb)
          const double* Rv = tall ? Vb[p] : Ub[p];
          const int ldr = tall ? kb[p] : kk;
          const double* Lv = tall ? Ub[p] : Vb[p];
          const int ldl = tall ? m1 : kb[p];
          g.push_back({Q0[p], Rv, F + pr[p].a2, m2, k, kk, m2, ldr, n, 0, 0, 1.0, 0.0});
          cb.push_back({Lv, ldl, F + pr[p].a1, n, m1, k, 1.0, 0.0, 0});
        }
        sc.push_back({F + pr[p].a1, n, m1, k, sb[p]});
      }
      gemm_batched(c, g);
      copy_batched(c, cb);
      scale_columns(c, sc);
    } else {
      LV.K = 0;
      LV.F.alloc(sizeof(double));
    }
    stats.weak_rank[l] = LV.K;
    if (!feats.empty() && records_on()) {
      std::vector<float> tg(np);
      for (int p = 0; p < np; ++p) tg[p] = (float)std::log1p((double)(needed[p] >= 0 ? needed[p] : cols[p]));
      records_add(feats, tg);
    }
    prev_sig = std::move(cur_sig);
    prev_k = LV.k;
    H2_HIP(hipStreamSynchronize(c.s));
    if (verbose())
      std::fprintf(stderr, "  [h2_build] level %d: rounds %d, range cols %d, rank %d, %.1f ms so far\n",
                   l, r, K0, LV.K, now_ms() - t_start);
    keep_factors(l, LV.k, LV.K, LV.F.as<double>(), n);
    c.scratch.clear();
    c.stage.reset();
    stats.time_ms[3] += now_ms() - t0;
  }

  // ---- leaf diagonal blocks from stacked identities
  t0 = now_ms();
  const int nleaf = 1 << L;
  const int mmax = t->max_leaf;
  std::vector<DevBuf> Ddiag(nleaf);
  {
    om_buf.reserve((size_t)n * mmax * sizeof(double));
    y_buf.reserve((size_t)n * mmax * sizeof(double));
    double* om = om_buf.as<double>();
    double* y = y_buf.as<double>();
    const int64_t tot = (int64_t)n * mmax;
    k_fill_diag<<<(unsigned)((tot + 255) / 256), 256, 0, c.s>>>(n, mmax, nleaf,
                                                                t->d_cstart.as<int32_t>() + cid(L, 0), om);
    H2_LAUNCH_CHECK();
    S.apply(c, mmax, om, y);
    subtract_levels(c, t, lv, L + 1, om, y, mmax);
    check_finite(c, y, tot, "diagonal samples");
    std::vector<SymDesc> sd(nleaf);
    for (int i = 0; i < nleaf; ++i) {
      const int m = t->csize[cid(L, i)];
      Ddiag[i].alloc((size_t)m * m * sizeof(double));
      sd[i] = {y + t->cstart[cid(L, i)], n, m, Ddiag[i].as<double>()};
    }
    auto* dsd = (SymDesc*)c.stage.put(sd.data(), sd.size() * sizeof(SymDesc), c.s);
    k_sym<<<nleaf, 256, 0, c.s>>>(dsd);
    H2_LAUNCH_CHECK();
    H2_HIP(hipStreamSynchronize(c.s));
    c.stage.reset();
  }
  stats.time_ms[4] = now_ms() - t0;

  // ================================================================== recompression
  t0 = now_ms();
  const double tau_c = tau;
  const int ncl = t->nclusters();
  auto pair_rank = [&](int l, int lev, int i) { return lv[l].k[(i >> (lev - l)) >> 1]; };
  auto Frows = [&](int l, int lev, int i) -> const double* {
    return lv[l].F.as<double>() + t->cstart[cid(lev, i)];
  };
  // far partners grouped by sibling level
  auto sib_level = [](int lev, int i, int j) {
    int s = 0;
    while ((i >> s) != (j >> s)) ++s;
    return lev - s + 1;
  };
  // (R1) downsweep: R^l_t (k x k, column-major) for every cluster t and l <= lev(t)
  std::map<std::tuple<int, int, int>, double*> R;   // (lev, i, l) -> k x k
  std::vector<DevBuf> Rstore;
  for (int lev = 1; lev <= L; ++lev) {
    std::vector<std::map<int, std::vector<int>>> by(1 << lev);
    for (auto [a, bb] : t->far[lev]) by[a][sib_level(lev, a, bb)].push_back(bb);
    // sizes of this level's stacks
    struct Job { int i, l, k, rows; double* stack; double* out; };
    std::vector<Job> jobs;
    int64_t total_out = 0, total_stack = 0;
    for (int i = 0; i < (1 << lev); ++i)
      for (int l = 1; l <= lev; ++l) {
        const int k = pair_rank(l, lev, i);
        if (k == 0) continue;
        auto it = by[i].find(l);
        const bool own = it != by[i].end();
        const bool par = l <= lev - 1 && R.count({lev - 1, i >> 1, l});
        if (!own && !par) continue;
        if (!own) {  // only the parent's block row: reuse its factor
          R[{lev, i, l}] = R[{lev - 1, i >> 1, l}];
          continue;
        }
        int rows = par ? k : 0;
        for (int j : it->second) rows += t->csize[cid(lev, j)];
        jobs.push_back({i, l, k, rows, nullptr, nullptr});
        total_out += (int64_t)k * k;
        total_stack += (int64_t)rows * k;
      }
    if (jobs.empty()) continue;
    Rstore.emplace_back(std::max<int64_t>(total_out, 1) * sizeof(double));
    H2_HIP(hipMemsetAsync(Rstore.back().p, 0, Rstore.back().bytes, c.s));
    DevBuf stack_buf(std::max<int64_t>(total_stack, 1) * sizeof(double));
    double* outp = Rstore.back().as<double>();
    double* stp = stack_buf.as<double>();
    std::vector<CopyDesc> cps;
    std::vector<QRDesc> qrs;
    for (auto& jb : jobs) {
      jb.out = outp;
      outp += (size_t)jb.k * jb.k;
      jb.stack = stp;
      stp += (size_t)jb.rows * jb.k;
      int row = 0;
      if (jb.l <= lev - 1 && R.count({lev - 1, jb.i >> 1, jb.l})) {
        cps.push_back({R[{lev - 1, jb.i >> 1, jb.l}], jb.k, jb.stack, jb.rows, jb.k, jb.k, 1.0, 0.0, 0});
        row += jb.k;
      }
      for (int j : by[jb.i][jb.l]) {
        const int mj = t->csize[cid(lev, j)];
        cps.push_back({Frows(jb.l, lev, j), n, jb.stack + row, jb.rows, mj, jb.k, 1.0, 0.0, 0});
        row += mj;
      }
      qrs.push_back({jb.stack, jb.rows, jb.rows, jb.k, nullptr, 0, jb.out, jb.k});
      R[{lev, jb.i, jb.l}] = jb.out;
    }
    copy_batched(c, cps);
    // R of a stack with fewer rows than k is min(rows,k) x k: ldr = k keeps the
    // zero rows below it (zeroed above)
    qr_auto(c, qrs);
    H2_HIP(hipStreamSynchronize(c.s));
    c.stage.reset();
  }

  // (R2) upsweep: bases, transfers, projections P^l_t = U_t^T F^l_t
  std::vector<int32_t> rank(ncl, 0);
  std::vector<DevBuf> Ubuf(nleaf), Ebuf(ncl);  // U: |t| x k col-major; E: (k1+k2) x k col-major
  std::map<std::pair<int, int>, std::vector<double*>> P;  // (lev, i) -> P^l, l = 1..lev
  std::vector<DevBuf> Pstore;
  bool cap_hit = false;
  for (int lev = L; lev >= 1; --lev) {
    const int nc = 1 << lev;
    std::vector<LsvTask> tasks;
    std::vector<int> Ms(nc), Ks(nc);
    std::vector<double*> Gs(nc), Us(nc), sg(nc);
    std::vector<GemmDesc> gg;
    std::vector<int64_t> goff(nc + 1, 0);
    for (int i = 0; i < nc; ++i) {
      const int M = lev == L ? t->csize[cid(L, i)] : rank[cid(lev + 1, 2 * i)] + rank[cid(lev + 1, 2 * i + 1)];
      int K = 0;
      for (int l = 1; l <= lev; ++l)
        if (R.count({lev, i, l})) K += pair_rank(l, lev, i);
      Ms[i] = M;
      Ks[i] = K;
      goff[i + 1] = goff[i] + std::min(M, K);
    }
    double* sg_all = c.scratch.get(std::max<int64_t>(goff[nc], 1));
    for (int i = 0; i < nc; ++i) {
      const int M = Ms[i], K = Ks[i];
      if (M == 0 || K == 0) continue;
      Gs[i] = c.scratch.get((size_t)M * K);
      int col = 0;
      for (int l = 1; l <= lev; ++l) {
        if (!R.count({lev, i, l})) continue;
        const int k = pair_rank(l, lev, i);
        double* Rl = R[{lev, i, l}];
        if (lev == L) {
          // G[:, col:col+k] = F^l_t R^T
          gg.push_back({Frows(l, L, i), Rl, Gs[i] + (size_t)col * M, M, k, k, n, k, M, 0, 1, 1.0, 0.0});
        } else {
          const int k1 = rank[cid(lev + 1, 2 * i)];
          const int k2 = rank[cid(lev + 1, 2 * i + 1)];
          if (k1) gg.push_back({P[{lev + 1, 2 * i}][l - 1], Rl, Gs[i] + (size_t)col * M, k1, k, k, k1, k, M, 0, 1, 1.0, 0.0});
          if (k2) gg.push_back({P[{lev + 1, 2 * i + 1}][l - 1], Rl, Gs[i] + (size_t)col * M + k1, k2, k, k, k2, k, M, 0, 1, 1.0, 0.0});
        }
        col += k;
      }
      const int r = std::min(M, K);
      Us[i] = c.scratch.get((size_t)M * r);
      sg[i] = sg_all + goff[i];
      tasks.push_back({Gs[i], M, M, K, Us[i], sg[i]});
    }
    gemm_batched(c, gg);
    left_svd_batched(c, tasks);
    // truncation (host decision)
    auto sgh = to_host(sg_all, goff[nc], c.s);
    for (int i = 0; i < nc; ++i) {
      int k = 0;
      if (Ms[i] > 0 && Ks[i] > 0) {
        const int r = std::min(Ms[i], Ks[i]);
        const double* s = sgh.data() + goff[i];
        H2_CHECK(std::isfinite(s[0]), H2_ENUMERIC, "non-finite singular values in recompression");
        while (k < r && s[k] > tau_c) ++k;
        if (k > prm.rank_cap) { k = prm.rank_cap; cap_hit = true; }
      }
      rank[cid(lev, i)] = k;
    }
    // keep the bases and compute the projections of this level
    int64_t ptot = 0;
    for (int i = 0; i < nc; ++i)
      for (int l = 1; l <= lev; ++l) ptot += (int64_t)rank[cid(lev, i)] * pair_rank(l, lev, i);
    Pstore.emplace_back(std::max<int64_t>(ptot, 1) * sizeof(double));
    double* pp = Pstore.back().as<double>();
    std::vector<GemmDesc> gp1, gp2;
    std::vector<CopyDesc> keep;
    for (int i = 0; i < nc; ++i) {
      const int k = rank[cid(lev, i)];
      const int M = Ms[i];
      auto& Pv = P[{lev, i}];
      Pv.assign(lev, nullptr);
      double* Ub = nullptr;
      if (lev == L) {
        Ubuf[i].alloc((size_t)std::max(M * k, 1) * sizeof(double));
        Ub = Ubuf[i].as<double>();
      } else {
        Ebuf[cid(lev, i)].alloc((size_t)std::max(M * k, 1) * sizeof(double));
        Ub = Ebuf[cid(lev, i)].as<double>();
      }
      if (k > 0) keep.push_back({Us[i], M, Ub, M, M, k, 1.0, 0.0, 0});
      for (int l = 1; l <= lev; ++l) {
        const int kl = pair_rank(l, lev, i);
        Pv[l - 1] = pp;
        pp += (size_t)k * kl;
        if (k == 0 || kl == 0) continue;
        if (lev == L) {
          // P = U^T F^l
          gp1.push_back({Us[i], Frows(l, L, i), Pv[l - 1], k, kl, M, M, n, k, 1, 0, 1.0, 0.0});
        } else {
          const int k1 = rank[cid(lev + 1, 2 * i)];
          const int k2 = rank[cid(lev + 1, 2 * i + 1)];
          // P = E1^T P1 + E2^T P2 with [E1; E2] = Us (M x k)
          if (k1) gp1.push_back({Us[i], P[{lev + 1, 2 * i}][l - 1], Pv[l - 1], k, kl, k1, M, k1, k, 1, 0, 1.0, 0.0});
          if (k2) gp2.push_back({Us[i] + k1, P[{lev + 1, 2 * i + 1}][l - 1], Pv[l - 1], k, kl, k2, M, k2, k, 1, 0, 1.0, k1 ? 1.0 : 0.0});
        }
      }
    }
    copy_batched(c, keep);
    gemm_batched(c, gp1);
    gemm_batched(c, gp2);
    H2_HIP(hipStreamSynchronize(c.s));
    c.scratch.clear();
    c.stage.reset();
  }
  stats.cap_hit = cap_hit;

  // ---- assemble the destination layout
  auto A = std::make_unique<h2_matrix>();
  matrix_layout(A.get(), t, rank);
  matrix_alloc(A.get(), H2_FP64);
  {
    std::vector<CopyDesc> cps;
    double* U = A->st.U.as<double>();
    for (int i = 0; i < nleaf; ++i) {
      const int k = rank[cid(L, i)], m = t->csize[cid(L, i)];
      // row-major |t| x k = column-major k x |t| = transpose of the basis
      if (k) cps.push_back({Ubuf[i].as<double>(), m, U + A->U_off[i], k, k, m, 1.0, 0.0, 1});
    }
    double* E = A->st.E.as<double>();
    for (int lev = 1; lev < L; ++lev)
      for (int i = 0; i < (1 << lev); ++i) {
        const int k = rank[cid(lev, i)];
        if (!k) continue;
        const int c1 = cid(lev + 1, 2 * i), c2 = c1 + 1;
        const int k1 = rank[c1], k2 = rank[c2], M = k1 + k2;
        const double* Eb = Ebuf[cid(lev, i)].as<double>();
        // E_c row-major (k_c x k) = column-major (k x k_c) = transpose of rows of Eb
        if (k1) cps.push_back({Eb, M, E + A->E_off[c1], k, k, k1, 1.0, 0.0, 1});
        if (k2) cps.push_back({Eb + k1, M, E + A->E_off[c2], k, k, k2, 1.0, 0.0, 1});
      }
    copy_batched(c, cps);
    // couplings S_ts = P^l_t (P^l_s)^T, stored row-major = column-major S^T = P_s P_t^T
    std::vector<GemmDesc> gs;
    double* Sd = A->st.S.as<double>();
    for (int lev = 1; lev <= L; ++lev)
      for (size_t q = 0; q < t->far[lev].size(); ++q) {
        auto [a, bb] = t->far[lev][q];
        const int64_t g = t->far_base[lev] + (int64_t)q;
        const int ka = rank[cid(lev, a)], kb = rank[cid(lev, bb)];
        if (!ka || !kb) continue;
        const int l = sib_level(lev, a, bb);
        const int kl = pair_rank(l, lev, a);
        gs.push_back({P[{lev, bb}][l - 1], P[{lev, a}][l - 1], Sd + A->S_off[g], kb, ka, kl, kb, ka, kb, 0, 1, 1.0, 0.0});
      }
    // dense near blocks D_ts = F^l_t (F^l_s)^T, row-major = column-major F_s F_t^T
    double* Dd = A->st.D.as<double>();
    std::vector<CopyDesc> diag_cps;
    for (size_t q = 0; q < t->near.size(); ++q) {
      auto [a, bb] = t->near[q];
      const int ma = t->csize[cid(L, a)], mb = t->csize[cid(L, bb)];
      if (a == bb) {
        diag_cps.push_back({Ddiag[a].as<double>(), ma, Dd + A->D_off[q], ma, ma, ma, 1.0, 0.0, 0});
        continue;
      }
      const int l = sib_level(L, a, bb);
      const int kl = pair_rank(l, L, a);
      if (kl == 0) {
        zero_block(c, Dd + A->D_off[q], mb, ma, mb);
        continue;
      }
      gs.push_back({Frows(l, L, bb), Frows(l, L, a), Dd + A->D_off[q], mb, ma, kl, n, n, mb, 0, 1, 1.0, 0.0});
    }
    // zero couplings with an empty side are sized 0; nothing to write
    copy_batched(c, diag_cps);
    gemm_batched(c, gs);
    H2_HIP(hipStreamSynchronize(c.s));
    c.scratch.clear();
    c.stage.reset();
  }
  stats.time_ms[5] = now_ms() - t0;
  for (int lev = 0; lev <= L; ++lev) {
    int mx = 0;
    for (int i = 0; i < (1 << lev); ++i) mx = std::max(mx, (int)rank[cid(lev, i)]);
    stats.strong_rank[lev] = mx;
  }
  stats.applies = S.applies - applies1;
  stats.converged = converged;
  stats.time_ms[7] = now_ms() - t_start;
  if (verbose())
    std::fprintf(stderr, "  [h2_build] done: applies %lld, ms norm %.1f sample %.1f range %.1f proj %.1f diag %.1f recompress %.1f total %.1f\n",
                 (long long)stats.applies, stats.time_ms[0], stats.time_ms[1], stats.time_ms[2],
                 stats.time_ms[3], stats.time_ms[4], stats.time_ms[5], stats.time_ms[7]);
  if (converged_out) *converged_out = converged;
  return A;
}

}  // namespace h2

// ------------------------------------------------------------------ C ABI
using namespace h2;

namespace h2 {
h2_status guarded_status(const std::function<void()>& f);
}

extern "C" {

void h2_opts_default(h2_opts* o) {
  if (!o) return;
  *o = h2_opts{};
  o->rank_cap = 32;
  o->oversample = 10;
  o->tol = 1e-4;
  o->adaptive = 1;
  o->max_rounds = 16;
  o->seed = 1;
  o->iteration = 0;
  o->norm = 0;
  o->prec = H2_FP64;
  o->learned = nullptr;
}

h2_status h2_build(const h2_tree* tree, h2_sampler_fn sampler, void* ctx, const h2_opts* opts,
                   hipStream_t stream, h2_matrix** out, h2_build_stats* stats) {
  bool conv = true;
  h2_status st = guarded_status([&] {
    H2_CHECK(tree && sampler && opts && out, H2_EINVAL, "null argument");
    H2_CHECK(opts->tol > 0 && opts->tol < 1, H2_EINVAL, "tol must be in (0, 1)");
    H2_CHECK(opts->prec == H2_FP64, H2_EINVAL, "construction runs in FP64; convert afterwards");
    BuildParams p;
    p.rank_cap = opts->rank_cap;
    p.oversample = opts->oversample;
    p.tol = opts->tol;
    p.adaptive = opts->adaptive != 0;
    p.max_rounds = opts->max_rounds;
    p.mlp = opts->learned;
    p.seed = opts->seed;
    p.iteration = opts->iteration;
    p.norm = opts->norm;
    Ctx c;
    c.s = stream;
    UserSampler S(tree, sampler, ctx);
    auto A = build_h2(tree, S, p, c, stats, &conv);
    *out = A.release();
  });
  if (st == H2_OK && !conv) return H2_ENOTCONVERGED;
  return st;
}

}  // extern "C"
