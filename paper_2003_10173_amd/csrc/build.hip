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

void PackedBatch::apply(Ctx& c,
                        const std::vector<std::tuple<int, int, const double*, double*>>& reqs) {
  if (reqs.empty()) return;
  const int nprob = (int)trees.size();
  const int64_t ld = off[nprob];
  int ncols = 0;
  for (const auto& r : reqs) ncols = std::max(ncols, std::get<1>(r));
  if (ncols <= 0) return;
  H2_CHECK(ld <= INT32_MAX, H2_EINVAL, "packed rows exceed the int range");
  om.reserve((size_t)ld * ncols * sizeof(double));
  y.reserve((size_t)ld * ncols * sizeof(double));
  double* O = om.as<double>();
  double* Y = y.as<double>();
  // inactive problems and columns beyond a problem's own count stay zero
  zero_block(c, O, (int)ld, ncols, (int)ld);
  std::vector<int32_t> active(nprob, 0);
  for (const auto& r : reqs) {
    const int i = std::get<0>(r), nc = std::get<1>(r);
    active[i] = 1;
    if (nc > 0) scatter_rows(trees[i], nc, 1.0, std::get<2>(r), trees[i]->n, 0.0, O + off[i], (int)ld, c.s);
  }
  const int rc = fn(ctx, nprob, off.data(), active.data(), ncols, O, (int)ld, Y, c.s);
  if (rc != 0) throw Error(H2_ECALLBACK, "batched sampler callback returned " + std::to_string(rc));
  H2_HIP(hipGetLastError());
  ++calls;
  for (const auto& r : reqs) {
    const int i = std::get<0>(r), nc = std::get<1>(r);
    if (nc > 0) gather_rows(trees[i], nc, Y + off[i], (int)ld, std::get<3>(r), trees[i]->n, c.s);
  }
}

void apply_requests(Ctx& c, const std::vector<ApplyReq>& reqs) {
  std::vector<PackedBatch*> order;
  std::map<PackedBatch*, std::vector<std::tuple<int, int, const double*, double*>>> groups;
  std::map<PackedBatch*, std::vector<Sampler*>> members;
  for (const auto& r : reqs) {
    if (r.ncols <= 0) continue;
    PackedBatch* b = r.S->batch();
    if (!b) {
      r.S->apply(c, r.ncols, r.om, r.y);
      continue;
    }
    if (!groups.count(b)) order.push_back(b);
    groups[b].push_back({r.S->batch_index(), r.ncols, r.om, r.y});
    members[b].push_back(r.S);
  }
  for (PackedBatch* b : order) {
    b->apply(c, groups[b]);
    auto& g = groups[b];
    for (size_t k = 0; k < g.size(); ++k) members[b][k]->applies += std::get<1>(g[k]);
  }
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

// Left singular vectors and singular values of X (M x K, column-major, ld):
// K >= 2M: QR of X^T, Jacobi on R^T (normalised columns); M <= K < 2M:
// Jacobi on X^T; K < M: QR then Jacobi on R^T.  Writes U (M x r,
// ld M) with r = min(M, K) and sigma (r).  X is destroyed.
struct LsvTask {
  double* X;
  int ld, M, K;
  double* U;      // M x min(M,K)
  double* sigma;  // min(M,K)
  double tol = 0.0;  // Jacobi tolerance (SVDDesc::tol)
};

// Jacobi tolerance of the SVDs of a build: samples known to FP32 precision
// (rank cut 1e-7 sigma_1) are orthogonalised to 1e-2 of their rank cut, far
// below the samples' own error; FP64 samples to the FP64 rounding level
static double svd_tol(const BuildParams& p) { return p.rank_cut > 1e-12 ? 1e-2 * p.rank_cut : 0.0; }

// Jacobi tolerance of the range-basis SVD.  Its only outputs that matter are
// the count of singular values above rank_cut sigma_1 and, when directions
// are cut, the kept span; the basis is otherwise used only through its span
// (the projection's truncation SVD absorbs any rotation of it).  One-sided
// Jacobi stopped at column cosines <= t leaves columns A = Q D with
// |Q^T Q - I| <= n t, so every column norm is its singular value to relative
// accuracy n t / 2 (Ostrowski), tiny ones included: t = 1e-8 (n <= 1024:
// 5e-6 relative) decides the count like the rounding-level tolerance, and a
// cut direction (below rank_cut sigma_1) keeps cosines <= 1e-8 with the
// kept ones.  (t = 1e-6 moved built operators by up to 4e-10 relative,
// through the kept span where directions were cut.)
static double range_svd_tol(const BuildParams& p) { return std::max(svd_tol(p), 1e-8); }

void left_svd_batched(Ctx& c, const std::vector<LsvTask>& tasks) {
  std::vector<CopyDesc> tr;
  std::vector<QRDesc> qrs;
  std::vector<SVDDesc> svs;
  std::vector<GemmDesc> back;
  std::vector<QRDesc> rq;       // R-only QR of X^T (K >= 2M)
  std::vector<CopyDesc> rtr;    // R -> R^T
  for (const auto& tk : tasks) {
    if (tk.M == 0 || tk.K == 0) continue;
    if (tk.K >= 2 * tk.M) {
      // X^T = Q R: the left singular vectors of X are those of R^T, taken as
      // the normalised columns of one-sided Jacobi on R^T (M x M rows instead
      // of K; only the leading vectors, above the truncation, are used)
      double* Xt = c.scratch.get((size_t)tk.K * tk.M);
      double* R = c.scratch.get((size_t)tk.M * tk.M);
      double* Rt = c.scratch.get((size_t)tk.M * tk.M);
      tr.push_back({tk.X, tk.ld, Xt, tk.K, tk.K, tk.M, 1.0, 0.0, 1});
      rq.push_back({Xt, tk.K, tk.K, tk.M, nullptr, 0, R, tk.M});
      rtr.push_back({R, tk.M, Rt, tk.M, tk.M, tk.M, 1.0, 0.0, 1});
      svs.push_back({Rt, tk.M, tk.M, tk.M, tk.sigma, tk.U, tk.M, nullptr, 0, tk.tol});
    } else if (tk.K >= tk.M) {
      double* Xt = c.scratch.get((size_t)tk.K * tk.M);
      tr.push_back({tk.X, tk.ld, Xt, tk.K, tk.K, tk.M, 1.0, 0.0, 1});
      svs.push_back({Xt, tk.K, tk.K, tk.M, tk.sigma, nullptr, 0, tk.U, tk.M, tk.tol});
    } else {
      double* Q = c.scratch.get((size_t)tk.M * tk.K);
      double* R = c.scratch.get((size_t)tk.K * tk.K);
      double* Rt = c.scratch.get((size_t)tk.K * tk.K);
      double* V = c.scratch.get((size_t)tk.K * tk.K);
      qrs.push_back({tk.X, tk.ld, tk.M, tk.K, Q, tk.M, R, tk.K});
      tr.push_back({R, tk.K, Rt, tk.K, tk.K, tk.K, 1.0, 0.0, 1});
      svs.push_back({Rt, tk.K, tk.K, tk.K, tk.sigma, nullptr, 0, V, tk.K, tk.tol});
      back.push_back({Q, V, tk.U, tk.M, tk.K, tk.K, tk.M, tk.K, tk.M, 0, 0, 1.0, 0.0});
    }
  }
  qr_auto(c, qrs);
  copy_batched(c, tr);
  qr_auto(c, rq);
  copy_batched(c, rtr);
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
namespace {

// per-problem state of a (batched) construction
struct JobState {
  BuildJob* J = nullptr;
  const h2_tree* t = nullptr;
  Sampler* S = nullptr;
  const BuildParams* prm = nullptr;
  int n = 0, L = 0, b = 0;
  double nu = 0, tau = 0;
  int64_t applies1 = 0;
  std::vector<Level> lv;
  std::vector<std::vector<double>> prev_sig;  // singular values of B0 per pair, previous level
  std::vector<int> prev_k;
  DevBuf om_buf, y_buf;
  // level l
  int np = 0;
  std::vector<Pair> pr;
  int b0 = 0, max_rounds = 0, cmax = 0, r = 0;
  bool sampling = false;
  std::vector<int64_t> zoff, qoff;
  DevBuf zbuf, qbuf, ebuf;
  double* Z = nullptr;
  double* Qe = nullptr;
  double* om = nullptr;
  double* y = nullptr;
  std::vector<int> cols, qc, needed, newly, act;
  std::vector<char> frozen;
  std::vector<float> feats;
  std::vector<double*> Yproj;
  // range basis and projection of level l
  std::vector<int> kq, k0, kb, mode;
  std::vector<double*> Vp, Q0, Ub, Vb, sb, QB;
  std::vector<int64_t> soff, boff;
  double* sig_all = nullptr;
  double* sb_all = nullptr;
  int K0 = 0;
  std::vector<std::vector<double>> cur_sig;
  // diagonal and recompression
  std::vector<DevBuf> Ddiag;
  std::map<std::tuple<int, int, int>, double*> R;  // (lev, i, l) -> k x k
  std::vector<DevBuf> Rstore;
  std::vector<int32_t> rank;
  std::vector<DevBuf> Ubuf, Ebuf;
  std::map<std::pair<int, int>, std::vector<double*>> P;  // (lev, i) -> P^l, l = 1..lev
  std::vector<DevBuf> Pstore;
  bool cap_hit = false;

  int pair_rank(int l, int lev, int i) const { return lv[l].k[(i >> (lev - l)) >> 1]; }
  const double* Frows(int l, int lev, int i) const {
    return lv[l].F.as<double>() + t->cstart[cid(lev, i)];
  }
};

int sib_level(int lev, int i, int j) {
  int s = 0;
  while ((i >> s) != (j >> s)) ++s;
  return lev - s + 1;
}

// Y -= sum_{l' < lmax} Atilde_{l'} Om for several problems: one launch pair
// (coefficients, update) per level l' across the problems
struct SubReq {
  const JobState* js;
  int lmax;
  const double* om;
  double* y;
  int ncols;
};
void subtract_multi(Ctx& c, const std::vector<SubReq>& reqs) {
  int lm = 0;
  for (auto& q : reqs) lm = std::max(lm, q.lmax);
  for (int l = 1; l < lm; ++l) {
    std::vector<GemmDesc> red, upd;
    for (auto& q : reqs) {
      if (l >= q.lmax) continue;
      const h2_tree* t = q.js->t;
      const Level& Lv = q.js->lv[l];
      if (Lv.K == 0) continue;
      const int n = t->n, ncols = q.ncols;
      const double* F = Lv.F.as<double>();
      for (int p = 0; p < (1 << (l - 1)); ++p) {
        const int k = Lv.k[p];
        if (k == 0) continue;
        const int a1 = t->cstart[cid(l, 2 * p)], m1 = t->csize[cid(l, 2 * p)];
        const int a2 = t->cstart[cid(l, 2 * p + 1)], m2 = t->csize[cid(l, 2 * p + 1)];
        double* c1 = c.scratch.get((size_t)k * ncols);
        double* c2 = c.scratch.get((size_t)k * ncols);
        red.push_back({F + a1, q.om + a1, c1, k, ncols, m1, n, n, k, 1, 0, 1.0, 0.0});
        red.push_back({F + a2, q.om + a2, c2, k, ncols, m2, n, n, k, 1, 0, 1.0, 0.0});
        upd.push_back({F + a2, c1, q.y + a2, m2, ncols, k, n, k, n, 0, 0, -1.0, 1.0});
        upd.push_back({F + a1, c2, q.y + a1, m1, ncols, k, n, k, n, 0, 0, -1.0, 1.0});
      }
    }
    gemm_batched(c, red);
    gemm_batched(c, upd);
  }
}

// one flag for several arrays: throws if any holds NaN/Inf
void check_finite_multi(Ctx& c, const std::vector<std::pair<const double*, int64_t>>& arrs,
                        const char* what) {
  DevBuf flag(sizeof(int));
  H2_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), c.s));
  for (auto& a : arrs)
    if (a.second > 0) {
      k_nonfinite<<<(unsigned)((a.second + 255) / 256), 256, 0, c.s>>>(a.second, a.first, flag.as<int>());
      H2_LAUNCH_CHECK();
    }
  int h = 0;
  H2_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, c.s));
  H2_HIP(hipStreamSynchronize(c.s));
  H2_CHECK(h == 0, H2_ENUMERIC, std::string("non-finite values in ") + what);
}

void set_pairs(JobState& s, int l) {
  const h2_tree* t = s.t;
  s.np = 1 << (l - 1);
  s.pr.assign(s.np, Pair{});
  for (int p = 0; p < s.np; ++p)
    s.pr[p] = {t->cstart[cid(l, 2 * p)], t->csize[cid(l, 2 * p)], t->cstart[cid(l, 2 * p + 1)],
               t->csize[cid(l, 2 * p + 1)]};
}

// first-round width (learned prediction or the plain width) and sample stores
void level_setup(JobState& s, int l, Ctx& c) {
  const BuildParams& prm = *s.prm;
  const int np = s.np, b = s.b, n = s.n;
  s.b0 = b;
  s.feats.clear();
  if (prm.adaptive && (prm.mlp || records_on()))
    s.feats = pair_features(s.t, l, prm.tol, s.prev_sig, s.prev_k);
  if (prm.adaptive && prm.mlp) {
    auto* dX = (float*)c.stage.put(s.feats.data(), s.feats.size() * sizeof(float), c.s);
    DevBuf dy((size_t)np * sizeof(float));
    mlp_forward(prm.mlp, np, dX, dy.as<float>(), c.s);
    std::vector<float> pred(np);
    H2_HIP(hipMemcpyAsync(pred.data(), dy.p, np * sizeof(float), hipMemcpyDeviceToHost, c.s));
    H2_HIP(hipStreamSynchronize(c.s));
    float ymax = -1e30f;
    for (float v : pred) {
      H2_CHECK(std::isfinite(v), H2_ENUMERIC, "non-finite rank prediction");
      ymax = std::max(ymax, v);
    }
    const double kpred = std::max(0.0, std::expm1((double)ymax));
    s.b0 = (int)std::min<double>(std::max<double>(b, std::ceil(kpred) + prm.oversample), 1024 - b);
    s.b0 = std::max(s.b0, b);
  }
  s.J->stats.first_cols[l] = s.b0;
  // the per-pair sample store holds at most 1024 columns (QR / SVD limit)
  s.max_rounds = std::max(2, std::min(prm.max_rounds, 1 + (1024 - s.b0) / b));
  s.cmax = prm.adaptive ? s.b0 + (s.max_rounds - 1) * b : b;
  // per-pair sample storage Z_p (m2 x cmax, ld m2) and an orthonormal basis
  // Qe_p of the samples kept so far (block Gram-Schmidt with two projections
  // per round), used by the estimator and by the final range basis
  s.zoff.assign(np + 1, 0);
  s.qoff.assign(np + 1, 0);
  for (int p = 0; p < np; ++p) {
    s.zoff[p + 1] = s.zoff[p] + (int64_t)s.pr[p].m2 * s.cmax;
    s.qoff[p + 1] = s.qoff[p] + (int64_t)s.pr[p].m2 * std::min(s.pr[p].m2, s.cmax);
  }
  s.zbuf.alloc(std::max<int64_t>(s.zoff[np], 1) * sizeof(double));
  s.qbuf.alloc(std::max<int64_t>(s.qoff[np], 1) * sizeof(double));
  s.Z = s.zbuf.as<double>();
  s.Qe = s.qbuf.as<double>();
  s.cols.assign(np, 0);
  s.qc.assign(np, 0);
  s.needed.assign(np, -1);
  s.frozen.assign(np, 0);
  s.om_buf.reserve((size_t)n * s.b0 * sizeof(double));
  s.y_buf.reserve((size_t)n * s.b0 * sizeof(double));
  s.om = s.om_buf.as<double>();
  s.y = s.y_buf.as<double>();
  s.ebuf.alloc(np * sizeof(double));
  s.r = 0;
  s.sampling = true;
}

}  // namespace

void build_h2_multi(std::vector<BuildJob>& jobs, Ctx& c) {
  const double t_start = now_ms();
  const double kHMT = 10.0 * std::sqrt(2.0 / M_PI);
  std::vector<JobState> js(jobs.size());
  int Lmax = 0;
  for (size_t j = 0; j < jobs.size(); ++j) {
    BuildJob& J = jobs[j];
    JobState& s = js[j];
    const BuildParams& prm = J.prm;
    H2_CHECK(J.t && J.S, H2_EINVAL, "build job without tree or sampler");
    s.J = &J;
    s.t = J.t;
    s.S = J.S;
    s.prm = &J.prm;
    s.n = J.t->n;
    s.L = J.t->L;
    s.b = prm.rank_cap + prm.oversample;
    H2_CHECK(s.b >= 1 && prm.rank_cap >= 1, H2_EINVAL, "rank_cap + oversample must be >= 1");
    H2_CHECK(!prm.adaptive || prm.max_rounds >= 2, H2_EINVAL, "adaptive mode needs max_rounds >= 2");
    H2_CHECK(s.b <= (prm.adaptive ? 512 : 1024), H2_EINVAL,
             "rank_cap + oversample must be <= 512 (adaptive) or 1024 (one round)");
    tree_device(J.t);
    J.stats = h2_build_stats{};
    J.stats.levels = s.L;
    J.converged = true;
    s.lv.resize(s.L + 1);
    Lmax = std::max(Lmax, s.L);
  }
  if (jobs.size() == 1) reset_factors();

  // ---- norm estimates (power method through each sampler, in lock step;
  // the products of one step go out as one request list)
  double t0 = now_ms();
  {
    std::vector<PowerJob> pj;
    std::vector<JobState*> pw;
    for (auto& s : js) {
      if (s.prm->norm > 0) continue;
      PowerJob J;
      J.n = s.n;
      J.seed = s.prm->seed;
      J.iteration = s.prm->iteration;
      J.rel = s.prm->norm_rel;
      J.min_it = 3;
      J.max_it = s.prm->norm_rel >= 1e-2 ? 30 : 500;
      pj.push_back(J);
      pw.push_back(&s);
    }
    for (auto* s : pw) s->applies1 = s->S->applies;
    if (!pj.empty()) {
      PowerBatchOp op = [&](const std::vector<int>& ids, const std::vector<const double*>& v,
                            const std::vector<double*>& w, hipStream_t) {
        std::vector<ApplyReq> reqs;
        for (size_t k = 0; k < ids.size(); ++k) reqs.push_back({pw[ids[k]]->S, 1, v[k], w[k]});
        apply_requests(c, reqs);
      };
      power_norm_multi(pj, c.s, false, &op);
    }
    for (size_t k = 0; k < pw.size(); ++k) pw[k]->nu = pj[k].result;
  }
  for (auto& s : js) {
    const BuildParams& prm = *s.prm;
    const int64_t a0 = prm.norm > 0 ? s.S->applies : s.applies1;
    double nu = prm.norm > 0 ? prm.norm : s.nu;
    H2_CHECK(std::isfinite(nu), H2_ENUMERIC, "norm estimate is not finite");
    s.nu = nu;
    s.J->stats.norm = nu;
    s.J->stats.norm_applies = s.S->applies - a0;
    s.applies1 = s.S->applies;
    s.tau = prm.tol * nu / (4.0 * std::max(s.L, 1));
  }
  const double t_norm = now_ms() - t0;
  double t_sample = 0, t_range = 0, t_proj = 0;

  for (int l = 1; l <= Lmax; ++l) {
    std::vector<JobState*> lj;  // problems that have level l
    for (auto& s : js)
      if (s.L >= l) lj.push_back(&s);
    for (JobState* s : lj) {
      set_pairs(*s, l);
      level_setup(*s, l, c);
    }
    c.stage.reset();
    t0 = now_ms();
    // ---- sampling rounds (problems keep sampling until their pairs converge)
    while (true) {
      std::vector<JobState*> sj;
      for (JobState* s : lj)
        if (s->sampling) sj.push_back(s);
      if (sj.empty()) break;
      std::vector<SubReq> sub;
      std::vector<ApplyReq> reqs;
      for (JobState* s : sj) {
        const int bw = s->r == 0 ? s->b0 : s->b;  // the first round may be wider (learned)
        const uint64_t key = stream_key(s->prm->seed, PHASE_RANGE, l, s->r, s->prm->iteration);
        const int64_t tot = (int64_t)s->n * bw;
        k_fill_left<<<(unsigned)((tot + 255) / 256), 256, 0, c.s>>>(
            key, s->n, bw, 1 << l, s->t->d_cstart.as<int32_t>() + cid(l, 0), s->om);
        H2_LAUNCH_CHECK();
        reqs.push_back({s->S, bw, s->om, s->y});
        sub.push_back({s, l, s->om, s->y, bw});
      }
      apply_requests(c, reqs);
      subtract_multi(c, sub);
      {
        std::vector<std::pair<const double*, int64_t>> fin;
        for (JobState* s : sj)
          if (s->r == 0) fin.push_back({s->y, (int64_t)s->n * s->b0});
        if (!fin.empty()) check_finite_multi(c, fin, "samples");
      }
      // projected samples Yp'' = (I - Qe Qe^T)^2 Y[t2] (round 0: the samples)
      {
        std::vector<CopyDesc> cp;
        std::vector<GemmDesc> g1, g2, g3, g4;
        for (JobState* s : sj) {
          const int bw = s->r == 0 ? s->b0 : s->b;
          s->newly.assign(s->np, 0);
          s->act.clear();
          for (int p = 0; p < s->np; ++p)
            if (!s->frozen[p]) s->act.push_back(p);
          s->Yproj.assign(s->np, nullptr);
          for (int p : s->act) {
            const int m2 = s->pr[p].m2;
            s->Yproj[p] = c.scratch.get((size_t)m2 * bw);
            cp.push_back({s->y + s->pr[p].a2, s->n, s->Yproj[p], m2, m2, bw, 1.0, 0.0, 0});
            const int q = s->qc[p];
            if (q == 0) continue;
            double* W1 = c.scratch.get((size_t)q * bw);
            double* W2 = c.scratch.get((size_t)q * bw);
            double* Qp_ = s->Qe + s->qoff[p];
            g1.push_back({Qp_, s->Yproj[p], W1, q, bw, m2, m2, m2, q, 1, 0, 1.0, 0.0});
            g2.push_back({Qp_, W1, s->Yproj[p], m2, bw, q, m2, q, m2, 0, 0, -1.0, 1.0});
            g3.push_back({Qp_, s->Yproj[p], W2, q, bw, m2, m2, m2, q, 1, 0, 1.0, 0.0});
            g4.push_back({Qp_, W2, s->Yproj[p], m2, bw, q, m2, q, m2, 0, 0, -1.0, 1.0});
          }
        }
        copy_batched(c, cp);
        gemm_batched(c, g1);
        gemm_batched(c, g2);
        gemm_batched(c, g3);
        gemm_batched(c, g4);
      }
      // estimator (rounds >= 1 of adaptive problems)
      {
        std::vector<CopyDesc> res_blocks;
        std::vector<std::pair<JobState*, int>> who;
        for (JobState* s : sj) {
          if (!s->prm->adaptive || s->r < 1) continue;
          const int bw = s->r == 0 ? s->b0 : s->b;
          for (int p : s->act) {
            res_blocks.push_back({s->Yproj[p], s->pr[p].m2, nullptr, 0, s->pr[p].m2, bw, 1.0, 0.0, 0});
            who.push_back({s, p});
          }
        }
        if (!res_blocks.empty()) {
          double* e_dev = c.scratch.get(res_blocks.size());
          colnorm_max_batched(c, res_blocks, e_dev);
          auto e = to_host(e_dev, res_blocks.size(), c.s);
          for (size_t q = 0; q < who.size(); ++q) {
            H2_CHECK(std::isfinite(e[q]), H2_ENUMERIC, "non-finite samples");
            JobState* s = who[q].first;
            const int p = who[q].second;
            if (kHMT * e[q] <= s->tau) {
              s->newly[p] = 1;
              s->needed[p] = s->cols[p];  // columns that sufficed, before this probe round
            }
          }
        }
      }
      // append this round's samples; extend Qe with the projected block: QR,
      // one more projection, QR again
      {
        std::vector<CopyDesc> app, put, lost;
        std::vector<uint64_t> lost_keys;
        std::vector<QRDesc> q1, q2, q3, t1, t2, t3;
        std::vector<GemmDesc> g1, g2, g3, g4;
        std::vector<size_t> t3_flag;   // lost-column flag of each t3 block
        for (JobState* s : sj) {
          const int bw = s->r == 0 ? s->b0 : s->b;
          for (int p : s->act) {
            const int m2 = s->pr[p].m2;
            app.push_back({s->y + s->pr[p].a2, s->n, s->Z + s->zoff[p] + (size_t)s->cols[p] * m2, m2,
                           m2, bw, 1.0, 0.0, 0});
            s->cols[p] += bw;
            const int q = s->qc[p];
            if (q >= m2) continue;
            const int kn = std::min(m2, bw);
            const int take = std::min(kn, m2 - q);
            const bool tall = m2 >= 2 * TSQR_MIN_ROWS && bw <= 96;  // else shape dispatch
            double* Qn = c.scratch.get((size_t)m2 * kn);
            double* Qn2 = c.scratch.get((size_t)m2 * kn);
            (tall ? t1 : q1).push_back({s->Yproj[p], m2, m2, bw, Qn, m2, nullptr, 0});
            if (q > 0) {
              double* Wq = c.scratch.get((size_t)q * kn);
              g1.push_back({s->Qe + s->qoff[p], Qn, Wq, q, kn, m2, m2, m2, q, 1, 0, 1.0, 0.0});
              g2.push_back({s->Qe + s->qoff[p], Wq, Qn, m2, kn, q, m2, q, m2, 0, 0, -1.0, 1.0});
              double* R2 = c.scratch.get((size_t)kn * kn);
              (tall ? t2 : q2).push_back({Qn, m2, m2, kn, Qn2, m2, R2, kn});
              // a round that adds fewer directions than columns (exactly
              // low-rank blocks) leaves columns of Qn2 dependent on Qe or on
              // each other (small R2_jj): they become Gaussian, are projected
              // once more and the block is orthonormalised again.  Blocks
              // with no such column skip these steps on the device (their
              // flag stays 0): the tall QR then runs in place on Qn2.
              const size_t fi = lost.size();
              lost.push_back({Qn2, m2, R2, kn, m2, kn, 1.0, 0.0, 0});
              lost_keys.push_back(stream_key(s->prm->seed, PHASE_LOST, (uint32_t)l,
                                             (uint32_t)(s->r * 4096 + p), s->prm->iteration));
              double* Wr = c.scratch.get((size_t)q * kn);
              g3.push_back({s->Qe + s->qoff[p], Qn2, Wr, q, kn, m2, m2, m2, q, 1, 0, 1.0, 0.0});
              g4.push_back({s->Qe + s->qoff[p], Wr, Qn2, m2, kn, q, m2, q, m2, 0, 0, -1.0, 1.0});
              double* Qn3 = tall ? Qn2 : c.scratch.get((size_t)m2 * kn);
              if (tall) {
                t3.push_back({Qn2, m2, m2, kn, Qn3, m2, nullptr, 0});
                t3_flag.push_back(fi);
              } else {
                q3.push_back({Qn2, m2, m2, kn, Qn3, m2, nullptr, 0});
              }
              put.push_back({Qn3, m2, s->Qe + s->qoff[p] + (size_t)q * m2, m2, m2, take, 1.0, 0.0, 0});
            } else {
              put.push_back({Qn, m2, s->Qe + s->qoff[p], m2, m2, take, 1.0, 0.0, 0});
            }
            s->qc[p] = q + take;
          }
        }
        copy_batched(c, app);
        qr_auto(c, q1);
        qr_tall_batched(c, t1);
        gemm_batched(c, g1);
        gemm_batched(c, g2);
        qr_auto(c, q2);
        qr_tall_batched(c, t2);
        int* flags = nullptr;
        if (!lost.empty()) {
          const int nd = (int)((lost.size() + 1) / 2);
          flags = (int*)c.scratch.get((size_t)nd);
          zero_block(c, (double*)flags, nd, 1, nd);
          for (size_t i = 0; i < lost.size(); ++i) {
            g3[i].run = flags + i;
            g4[i].run = flags + i;
          }
          for (size_t i = 0; i < t3.size(); ++i) t3[i].run = flags + t3_flag[i];
        }
        replace_lost_columns(c, lost, lost_keys, flags);
        gemm_batched(c, g3);
        gemm_batched(c, g4);
        qr_auto(c, q3);
        qr_tall_batched(c, t3);
        copy_batched(c, put);
      }
      H2_HIP(hipStreamSynchronize(c.s));
      c.scratch.clear();
      c.stage.reset();
      for (JobState* s : sj) {
        for (int p = 0; p < s->np; ++p)
          if (s->newly[p]) s->frozen[p] = 1;
        ++s->r;
        if (!s->prm->adaptive) { s->sampling = false; continue; }
        bool all = true;
        for (int p = 0; p < s->np; ++p) all = all && s->frozen[p];
        if (s->r >= 2 && all) s->sampling = false;
        else if (s->r >= s->max_rounds) {
          s->J->converged = false;
          s->sampling = false;
        }
      }
    }
    for (JobState* s : lj) s->J->stats.rounds[l] = s->r;
    t_sample += now_ms() - t0;

    // ---- range basis: Z = Qe (Qe^T Z); SVD of Qe^T Z, singular values above
    // rank_cut sigma_1 (the left singular vectors of the samples)
    t0 = now_ms();
    {
      std::vector<GemmDesc> g;
      std::vector<SVDDesc> svs;
      for (JobState* s : lj) {
        const int np = s->np;
        s->kq.assign(np, 0);
        s->k0.assign(np, 0);
        s->Vp.assign(np, nullptr);
        s->soff.assign(np + 1, 0);
        for (int p = 0; p < np; ++p) s->soff[p + 1] = s->soff[p] + s->qc[p];
        s->sig_all = c.scratch.get(std::max<int64_t>(s->soff[np], 1));
        for (int p = 0; p < np; ++p) {
          const int m2 = s->pr[p].m2, cp = s->cols[p];
          s->kq[p] = s->qc[p];
          // Rt = Z^T Qe (cp x kq) = (Qe^T Z)^T
          double* Rt = c.scratch.get((size_t)cp * s->kq[p]);
          s->Vp[p] = c.scratch.get((size_t)s->kq[p] * s->kq[p]);
          g.push_back({s->Z + s->zoff[p], s->Qe + s->qoff[p], Rt, cp, s->kq[p], m2, m2, m2, cp, 1, 0,
                       1.0, 0.0});
          // left singular vectors of R = right singular vectors of R^T
          svs.push_back({Rt, cp, cp, s->kq[p], s->sig_all + s->soff[p], nullptr, 0, s->Vp[p], s->kq[p],
                         range_svd_tol(*s->prm)});
        }
      }
      gemm_batched(c, g);
      svd_batched(c, svs);
    }
    {
      std::vector<GemmDesc> g;
      std::vector<CopyDesc> cs;
      H2_HIP(hipStreamSynchronize(c.s));
      for (JobState* s : lj) {
        const int np = s->np;
        auto sh = to_host(s->sig_all, s->soff[np], c.s);
        s->Q0.assign(np, nullptr);
        s->K0 = 0;
        for (int p = 0; p < np; ++p) {
          const double* sv = sh.data() + s->soff[p];
          int k = 0;
          if (s->kq[p] > 0 && sv[0] > 0) {
            H2_CHECK(std::isfinite(sv[0]), H2_ENUMERIC, "non-finite singular values");
            while (k < s->kq[p] && sv[k] > s->prm->rank_cut * sv[0]) ++k;
          }
          s->k0[p] = k;
          s->K0 = std::max(s->K0, k);
          if (verbose() && s->kq[p] >= 24)
            std::fprintf(stderr, "    [range] kq %d k0 %d smallest/largest %.2e\n", s->kq[p], k,
                         s->kq[p] > 0 && sv[0] > 0 ? sv[s->kq[p] - 1] / sv[0] : 0.0);
          const int m2 = s->pr[p].m2;
          s->Q0[p] = c.scratch.get((size_t)m2 * std::max(k, 1));
          if (k > 0) {
            g.push_back({s->Qe + s->qoff[p], s->Vp[p], s->Q0[p], m2, k, s->kq[p], m2, s->kq[p], m2, 0, 0,
                         1.0, 0.0});
            // canonical column signs: the projection below carries every pair's
            // basis in the same columns, so the result must not depend on signs
            cs.push_back({s->Q0[p], m2, nullptr, 0, m2, k, 1.0, 0.0, 0});
          }
        }
        s->J->stats.range_cols[l] = s->K0;
      }
      gemm_batched(c, g);
      canonical_signs(c, cs);
    }
    H2_HIP(hipStreamSynchronize(c.s));
    for (JobState* s : lj) {
      s->zbuf.release();
      s->qbuf.release();
    }
    t_range += now_ms() - t0;

    // ---- projection B0 = (A [0; Q0])[t1] and truncation
    t0 = now_ms();
    {
      std::vector<SubReq> sub;
      std::vector<ApplyReq> reqs;
      for (JobState* s : lj) {
        Level& LV = s->lv[l];
        LV.k.assign(s->np, 0);
        s->cur_sig.assign(s->np, {});
        if (s->K0 == 0) continue;
        const int n = s->n;
        s->om_buf.reserve((size_t)n * s->K0 * sizeof(double));
        s->y_buf.reserve((size_t)n * s->K0 * sizeof(double));
        s->om = s->om_buf.as<double>();
        s->y = s->y_buf.as<double>();
        zero_block(c, s->om, n, s->K0, n);
        std::vector<CopyDesc> put;
        for (int p = 0; p < s->np; ++p)
          if (s->k0[p] > 0)
            put.push_back({s->Q0[p], s->pr[p].m2, s->om + s->pr[p].a2, n, s->pr[p].m2, s->k0[p], 1.0, 0.0, 0});
        copy_batched(c, put);
        reqs.push_back({s->S, s->K0, s->om, s->y});
        sub.push_back({s, l, s->om, s->y, s->K0});
      }
      apply_requests(c, reqs);
      subtract_multi(c, sub);
    }
    // truncated SVD of B0 (m1 x k0) by one-sided Jacobi:
    //   mode 0 (m1 >= k0, small k0): B0 V = U S         -> Q = Q0 V_k, B = U_k S_k
    //   mode 1 (m1 <  k0):  B0^T V = U S, B0 = V S U^T  -> Q = Q0 U_k, B = V_k S_k
    //   mode 2 (m1 >= k0, large k0): B0 = Q_B R (blocked QR), R^T V = U S,
    //          B0 = (Q_B V) S U^T                        -> Q = Q0 U_k, B = Q_B V_k S_k
    {
      std::vector<CopyDesc> b0c, rtc;
      std::vector<CholQRDesc> bqr;
      std::vector<SVDDesc> svs;
      for (JobState* s : lj) {
        const int np = s->np, n = s->n;
        s->kb.assign(np, 0);
        s->mode.assign(np, 0);
        s->Ub.assign(np, nullptr);
        s->Vb.assign(np, nullptr);
        s->sb.assign(np, nullptr);
        s->QB.assign(np, nullptr);
        s->boff.assign(np + 1, 0);
        if (s->K0 == 0) continue;
        for (int p = 0; p < np; ++p) s->boff[p + 1] = s->boff[p] + std::min(s->pr[p].m1, s->k0[p]);
        s->sb_all = c.scratch.get(std::max<int64_t>(s->boff[np], 1));
        for (int p = 0; p < np; ++p) {
          if (s->k0[p] == 0) continue;
          const int m1 = s->pr[p].m1, kk = s->k0[p];
          s->kb[p] = std::min(m1, kk);
          s->sb[p] = s->sb_all + s->boff[p];
          if (m1 >= kk && kk >= 96 && m1 >= 128) {
            s->mode[p] = 2;
            s->QB[p] = c.scratch.get((size_t)m1 * kk);
            double* RB = c.scratch.get((size_t)kk * kk);
            double* RBt = c.scratch.get((size_t)kk * kk);
            b0c.push_back({s->y + s->pr[p].a1, n, s->QB[p], m1, m1, kk, 1.0, 0.0, 0});
            bqr.push_back({s->QB[p], m1, m1, kk, RB, kk});
            rtc.push_back({RB, kk, RBt, kk, kk, kk, 1.0, 0.0, 1});
            s->Ub[p] = c.scratch.get((size_t)kk * kk);
            s->Vb[p] = c.scratch.get((size_t)kk * kk);
            svs.push_back({RBt, kk, kk, kk, s->sb[p], s->Ub[p], kk, s->Vb[p], kk, svd_tol(*s->prm)});
            continue;
          }
          const bool tall = m1 >= kk;
          s->mode[p] = tall ? 0 : 1;
          const int mm = tall ? m1 : kk, nn = tall ? kk : m1;
          double* X = c.scratch.get((size_t)mm * nn);
          // a transposed copy reads B0 (m1 x k0 at y + a1, ld n) as its source
          b0c.push_back({s->y + s->pr[p].a1, n, X, mm, mm, nn, 1.0, 0.0, tall ? 0 : 1});
          s->Ub[p] = c.scratch.get((size_t)mm * nn);
          s->Vb[p] = c.scratch.get((size_t)nn * nn);
          svs.push_back({X, mm, mm, nn, s->sb[p], s->Ub[p], mm, s->Vb[p], nn, svd_tol(*s->prm)});
        }
      }
      copy_batched(c, b0c);
      qr_blocked(c, bqr);
      copy_batched(c, rtc);
      svd_batched(c, svs);
    }
    {
      std::vector<GemmDesc> g;
      std::vector<CopyDesc> cb;
      std::vector<ScaleDesc> sc;
      H2_HIP(hipStreamSynchronize(c.s));
      for (JobState* s : lj) {
        Level& LV = s->lv[l];
        const int np = s->np, n = s->n;
        if (s->K0 == 0) {
          LV.K = 0;
          LV.F.alloc(sizeof(double));
          continue;
        }
        auto sbh = to_host(s->sb_all, s->boff[np], c.s);
        for (int p = 0; p < np; ++p)
          s->cur_sig[p].assign(sbh.data() + s->boff[p], sbh.data() + s->boff[p] + s->kb[p]);
        for (int p = 0; p < np; ++p) {
          if (s->k0[p] == 0) continue;
          const double* sv = sbh.data() + s->boff[p];
          int k = 0;
          while (k < s->kb[p] && sv[k] > s->tau) ++k;
          H2_CHECK(s->kb[p] == 0 || std::isfinite(sv[0]), H2_ENUMERIC, "non-finite singular values");
          LV.k[p] = k;
        }
        LV.K = *std::max_element(LV.k.begin(), LV.k.end());
        LV.F.alloc((size_t)n * std::max(LV.K, 1) * sizeof(double));
        double* F = LV.F.as<double>();
        zero_block(c, F, n, std::max(LV.K, 1), n);
        for (int p = 0; p < np; ++p) {
          const int k = LV.k[p];
          if (k == 0) continue;
          const Pair& q = s->pr[p];
          const int m1 = q.m1, m2 = q.m2, kk = s->k0[p];
          if (s->mode[p] == 2) {
            g.push_back({s->Q0[p], s->Ub[p], F + q.a2, m2, k, kk, m2, kk, n, 0, 0, 1.0, 0.0});
            g.push_back({s->QB[p], s->Vb[p], F + q.a1, m1, k, kk, m1, kk, n, 0, 0, 1.0, 0.0});
          } else {
            const bool tall = s->mode[p] == 0;
            // right singular vectors of B0 (k0 x kb) and left ones (m1 x kb)
            const double* Rv = tall ? s->Vb[p] : s->Ub[p];
            const int ldr = tall ? s->kb[p] : kk;
            const double* Lv = tall ? s->Ub[p] : s->Vb[p];
            const int ldl = tall ? m1 : s->kb[p];
            g.push_back({s->Q0[p], Rv, F + q.a2, m2, k, kk, m2, ldr, n, 0, 0, 1.0, 0.0});
            cb.push_back({Lv, ldl, F + q.a1, n, m1, k, 1.0, 0.0, 0});
          }
          sc.push_back({F + q.a1, n, m1, k, s->sb[p]});
        }
      }
      gemm_batched(c, g);
      copy_batched(c, cb);
      scale_columns(c, sc);
    }
    for (JobState* s : lj) {
      Level& LV = s->lv[l];
      s->J->stats.weak_rank[l] = LV.K;
      if (!s->feats.empty() && records_on()) {
        std::vector<float> tg(s->np);
        for (int p = 0; p < s->np; ++p)
          tg[p] = (float)std::log1p((double)(s->needed[p] >= 0 ? s->needed[p] : s->cols[p]));
        records_add(s->feats, tg);
      }
      s->prev_sig = std::move(s->cur_sig);
      s->prev_k = LV.k;
    }
    H2_HIP(hipStreamSynchronize(c.s));
    if (verbose()) {
      int rmax = 0, k0m = 0, km = 0;
      for (JobState* s : lj) {
        rmax = std::max(rmax, s->r);
        k0m = std::max(k0m, s->K0);
        km = std::max(km, s->lv[l].K);
      }
      std::fprintf(stderr, "  [h2_build] level %d: %zu problems, rounds %d, range cols %d, rank %d, %.1f ms so far\n",
                   l, lj.size(), rmax, k0m, km, now_ms() - t_start);
    }
    if (jobs.size() == 1) {
      const JobState& s = js[0];
      keep_factors(l, s.lv[l].k, s.lv[l].K, s.lv[l].F.as<double>(), s.n);
    }
    c.scratch.clear();
    c.stage.reset();
    t_proj += now_ms() - t0;
  }

  // ---- leaf diagonal blocks from stacked identities
  t0 = now_ms();
  {
    std::vector<SubReq> sub;
    std::vector<std::pair<const double*, int64_t>> fin;
    std::vector<SymDesc> sd;
    std::vector<ApplyReq> reqs;
    for (auto& s : js) {
      const int n = s.n, L = s.L, nleaf = 1 << L, mmax = s.t->max_leaf;
      s.om_buf.reserve((size_t)n * mmax * sizeof(double));
      s.y_buf.reserve((size_t)n * mmax * sizeof(double));
      s.om = s.om_buf.as<double>();
      s.y = s.y_buf.as<double>();
      const int64_t tot = (int64_t)n * mmax;
      k_fill_diag<<<(unsigned)((tot + 255) / 256), 256, 0, c.s>>>(
          n, mmax, nleaf, s.t->d_cstart.as<int32_t>() + cid(L, 0), s.om);
      H2_LAUNCH_CHECK();
      reqs.push_back({s.S, mmax, s.om, s.y});
      sub.push_back({&s, L + 1, s.om, s.y, mmax});
      fin.push_back({s.y, tot});
      s.Ddiag.resize(nleaf);
      for (int i = 0; i < nleaf; ++i) {
        const int m = s.t->csize[cid(L, i)];
        s.Ddiag[i].alloc((size_t)m * m * sizeof(double));
        sd.push_back({s.y + s.t->cstart[cid(L, i)], n, m, s.Ddiag[i].as<double>()});
      }
    }
    apply_requests(c, reqs);
    subtract_multi(c, sub);
    check_finite_multi(c, fin, "diagonal samples");
    auto* dsd = (SymDesc*)c.stage.put(sd.data(), sd.size() * sizeof(SymDesc), c.s);
    k_sym<<<(unsigned)sd.size(), 256, 0, c.s>>>(dsd);
    H2_LAUNCH_CHECK();
    H2_HIP(hipStreamSynchronize(c.s));
    c.stage.reset();
  }
  const double t_diag = now_ms() - t0;

  // ================================================================== recompression
  t0 = now_ms();
  // (R1) downsweep: R^l_t (k x k, column-major) for every cluster t and l <= lev(t)
  for (int lev = 1; lev <= Lmax; ++lev) {
    std::vector<CopyDesc> cps;
    std::vector<QRDesc> qrs;
    std::vector<DevBuf> stacks;
    for (auto& s : js) {
      if (s.L < lev) continue;
      const h2_tree* t = s.t;
      std::vector<std::map<int, std::vector<int>>> by(1 << lev);
      for (auto [a, bb] : t->far[lev]) by[a][sib_level(lev, a, bb)].push_back(bb);
      struct Job { int i, l, k, rows; };
      std::vector<Job> jb;
      int64_t total_out = 0, total_stack = 0;
      for (int i = 0; i < (1 << lev); ++i)
        for (int l = 1; l <= lev; ++l) {
          const int k = s.pair_rank(l, lev, i);
          if (k == 0) continue;
          auto it = by[i].find(l);
          const bool own = it != by[i].end();
          const bool par = l <= lev - 1 && s.R.count({lev - 1, i >> 1, l});
          if (!own && !par) continue;
          if (!own) {  // only the parent's block row: reuse its factor
            s.R[{lev, i, l}] = s.R[{lev - 1, i >> 1, l}];
            continue;
          }
          int rows = par ? k : 0;
          for (int j : it->second) rows += t->csize[cid(lev, j)];
          jb.push_back({i, l, k, rows});
          total_out += (int64_t)k * k;
          total_stack += (int64_t)rows * k;
        }
      if (jb.empty()) continue;
      s.Rstore.emplace_back(std::max<int64_t>(total_out, 1) * sizeof(double));
      // R of a stack with fewer rows than k is min(rows,k) x k: ldr = k keeps
      // the zero rows below it
      zero_block(c, s.Rstore.back().as<double>(), (int)std::max<int64_t>(total_out, 1), 1,
                 (int)std::max<int64_t>(total_out, 1));
      stacks.emplace_back(std::max<int64_t>(total_stack, 1) * sizeof(double));
      double* outp = s.Rstore.back().as<double>();
      double* stp = stacks.back().as<double>();
      for (auto& q : jb) {
        double* out = outp;
        outp += (size_t)q.k * q.k;
        double* stack = stp;
        stp += (size_t)q.rows * q.k;
        int row = 0;
        if (q.l <= lev - 1 && s.R.count({lev - 1, q.i >> 1, q.l})) {
          cps.push_back({s.R[{lev - 1, q.i >> 1, q.l}], q.k, stack, q.rows, q.k, q.k, 1.0, 0.0, 0});
          row += q.k;
        }
        for (int j : by[q.i][q.l]) {
          const int mj = t->csize[cid(lev, j)];
          cps.push_back({s.Frows(q.l, lev, j), s.n, stack + row, q.rows, mj, q.k, 1.0, 0.0, 0});
          row += mj;
        }
        qrs.push_back({stack, q.rows, q.rows, q.k, nullptr, 0, out, q.k});
        s.R[{lev, q.i, q.l}] = out;
      }
    }
    copy_batched(c, cps);
    qr_auto(c, qrs);
    H2_HIP(hipStreamSynchronize(c.s));
    c.scratch.clear();
    c.stage.reset();
  }

  // (R2) upsweep: bases, transfers, projections P^l_t = U_t^T F^l_t
  for (auto& s : js) {
    s.rank.assign(s.t->nclusters(), 0);
    s.Ubuf.resize(1 << s.L);
    s.Ebuf.resize(s.t->nclusters());
  }
  for (int lev = Lmax; lev >= 1; --lev) {
    std::vector<LsvTask> tasks;
    std::vector<GemmDesc> gg;
    struct Up {
      JobState* s;
      std::vector<int> Ms, Ks;
      std::vector<double*> Us;
      std::vector<int64_t> goff;
      double* sg_all;
    };
    std::vector<Up> ups;
    for (auto& s : js) {
      if (s.L < lev) continue;
      const h2_tree* t = s.t;
      const int nc = 1 << lev, L = s.L, n = s.n;
      Up u{&s, std::vector<int>(nc), std::vector<int>(nc), std::vector<double*>(nc, nullptr),
           std::vector<int64_t>(nc + 1, 0), nullptr};
      for (int i = 0; i < nc; ++i) {
        const int M = lev == L ? t->csize[cid(L, i)]
                               : s.rank[cid(lev + 1, 2 * i)] + s.rank[cid(lev + 1, 2 * i + 1)];
        int K = 0;
        for (int l = 1; l <= lev; ++l)
          if (s.R.count({lev, i, l})) K += s.pair_rank(l, lev, i);
        u.Ms[i] = M;
        u.Ks[i] = K;
        u.goff[i + 1] = u.goff[i] + std::min(M, K);
      }
      u.sg_all = c.scratch.get(std::max<int64_t>(u.goff[nc], 1));
      for (int i = 0; i < nc; ++i) {
        const int M = u.Ms[i], K = u.Ks[i];
        if (M == 0 || K == 0) continue;
        double* G = c.scratch.get((size_t)M * K);
        int col = 0;
        for (int l = 1; l <= lev; ++l) {
          if (!s.R.count({lev, i, l})) continue;
          const int k = s.pair_rank(l, lev, i);
          double* Rl = s.R[{lev, i, l}];
          if (lev == L) {
            // G[:, col:col+k] = F^l_t R^T
            gg.push_back({s.Frows(l, L, i), Rl, G + (size_t)col * M, M, k, k, n, k, M, 0, 1, 1.0, 0.0});
          } else {
            const int k1 = s.rank[cid(lev + 1, 2 * i)];
            const int k2 = s.rank[cid(lev + 1, 2 * i + 1)];
            if (k1) gg.push_back({s.P[{lev + 1, 2 * i}][l - 1], Rl, G + (size_t)col * M, k1, k, k, k1, k, M, 0, 1, 1.0, 0.0});
            if (k2) gg.push_back({s.P[{lev + 1, 2 * i + 1}][l - 1], Rl, G + (size_t)col * M + k1, k2, k, k, k2, k, M, 0, 1, 1.0, 0.0});
          }
          col += k;
        }
        u.Us[i] = c.scratch.get((size_t)M * std::min(M, K));
        tasks.push_back({G, M, M, K, u.Us[i], u.sg_all + u.goff[i], svd_tol(*s.prm)});
      }
      ups.push_back(std::move(u));
    }
    gemm_batched(c, gg);
    left_svd_batched(c, tasks);
    H2_HIP(hipStreamSynchronize(c.s));
    std::vector<GemmDesc> gp1, gp2;
    std::vector<CopyDesc> keep;
    for (auto& u : ups) {
      JobState& s = *u.s;
      const h2_tree* t = s.t;
      const int nc = 1 << lev, L = s.L, n = s.n;
      // truncation (host decision)
      auto sgh = to_host(u.sg_all, u.goff[nc], c.s);
      for (int i = 0; i < nc; ++i) {
        int k = 0;
        if (u.Ms[i] > 0 && u.Ks[i] > 0) {
          const int r = std::min(u.Ms[i], u.Ks[i]);
          const double* sv = sgh.data() + u.goff[i];
          H2_CHECK(std::isfinite(sv[0]), H2_ENUMERIC, "non-finite singular values in recompression");
          while (k < r && sv[k] > s.tau) ++k;
          const int cap = s.prm->dest_cap > 0 ? s.prm->dest_cap : s.prm->rank_cap;
          if (k > cap) { k = cap; s.cap_hit = true; }
        }
        s.rank[cid(lev, i)] = k;
      }
      // keep the bases and compute the projections of this level
      int64_t ptot = 0;
      for (int i = 0; i < nc; ++i)
        for (int l = 1; l <= lev; ++l) ptot += (int64_t)s.rank[cid(lev, i)] * s.pair_rank(l, lev, i);
      s.Pstore.emplace_back(std::max<int64_t>(ptot, 1) * sizeof(double));
      double* pp = s.Pstore.back().as<double>();
      for (int i = 0; i < nc; ++i) {
        const int k = s.rank[cid(lev, i)];
        const int M = u.Ms[i];
        auto& Pv = s.P[{lev, i}];
        Pv.assign(lev, nullptr);
        double* Ub = nullptr;
        if (lev == L) {
          s.Ubuf[i].alloc((size_t)std::max(M * k, 1) * sizeof(double));
          Ub = s.Ubuf[i].as<double>();
        } else {
          s.Ebuf[cid(lev, i)].alloc((size_t)std::max(M * k, 1) * sizeof(double));
          Ub = s.Ebuf[cid(lev, i)].as<double>();
        }
        if (k > 0) keep.push_back({u.Us[i], M, Ub, M, M, k, 1.0, 0.0, 0});
        for (int l = 1; l <= lev; ++l) {
          const int kl = s.pair_rank(l, lev, i);
          Pv[l - 1] = pp;
          pp += (size_t)k * kl;
          if (k == 0 || kl == 0) continue;
          if (lev == L) {
            // P = U^T F^l
            gp1.push_back({u.Us[i], s.Frows(l, L, i), Pv[l - 1], k, kl, M, M, n, k, 1, 0, 1.0, 0.0});
          } else {
            const int k1 = s.rank[cid(lev + 1, 2 * i)];
            const int k2 = s.rank[cid(lev + 1, 2 * i + 1)];
            // P = E1^T P1 + E2^T P2 with [E1; E2] = Us (M x k)
            if (k1) gp1.push_back({u.Us[i], s.P[{lev + 1, 2 * i}][l - 1], Pv[l - 1], k, kl, k1, M, k1, k, 1, 0, 1.0, 0.0});
            if (k2) gp2.push_back({u.Us[i] + k1, s.P[{lev + 1, 2 * i + 1}][l - 1], Pv[l - 1], k, kl, k2, M, k2, k, 1, 0, 1.0, k1 ? 1.0 : 0.0});
          }
        }
      }
      (void)t;
    }
    copy_batched(c, keep);
    gemm_batched(c, gp1);
    gemm_batched(c, gp2);
    H2_HIP(hipStreamSynchronize(c.s));
    c.scratch.clear();
    c.stage.reset();
  }

  // ---- assemble the destination layouts
  {
    std::vector<CopyDesc> cps, diag_cps;
    std::vector<GemmDesc> gs;
    for (auto& s : js) {
      const h2_tree* t = s.t;
      const int L = s.L, n = s.n, nleaf = 1 << L;
      s.J->stats.cap_hit = s.cap_hit;
      auto A = std::make_unique<h2_matrix>();
      matrix_layout(A.get(), t, s.rank);
      matrix_alloc(A.get(), H2_FP64);
      double* U = A->st.U.as<double>();
      for (int i = 0; i < nleaf; ++i) {
        const int k = s.rank[cid(L, i)], m = t->csize[cid(L, i)];
        // row-major |t| x k = column-major k x |t| = transpose of the basis
        if (k) cps.push_back({s.Ubuf[i].as<double>(), m, U + A->U_off[i], k, k, m, 1.0, 0.0, 1});
      }
      double* E = A->st.E.as<double>();
      for (int lev = 1; lev < L; ++lev)
        for (int i = 0; i < (1 << lev); ++i) {
          const int k = s.rank[cid(lev, i)];
          if (!k) continue;
          const int c1 = cid(lev + 1, 2 * i), c2 = c1 + 1;
          const int k1 = s.rank[c1], k2 = s.rank[c2], M = k1 + k2;
          const double* Eb = s.Ebuf[cid(lev, i)].as<double>();
          // E_c row-major (k_c x k) = column-major (k x k_c) = transpose of rows of Eb
          if (k1) cps.push_back({Eb, M, E + A->E_off[c1], k, k, k1, 1.0, 0.0, 1});
          if (k2) cps.push_back({Eb + k1, M, E + A->E_off[c2], k, k, k2, 1.0, 0.0, 1});
        }
      // couplings S_ts = P^l_t (P^l_s)^T, stored row-major = column-major S^T = P_s P_t^T
      double* Sd = A->st.S.as<double>();
      for (int lev = 1; lev <= L; ++lev)
        for (size_t q = 0; q < t->far[lev].size(); ++q) {
          auto [a, bb] = t->far[lev][q];
          const int64_t g = t->far_base[lev] + (int64_t)q;
          const int ka = s.rank[cid(lev, a)], kb = s.rank[cid(lev, bb)];
          if (!ka || !kb) continue;
          const int l = sib_level(lev, a, bb);
          const int kl = s.pair_rank(l, lev, a);
          gs.push_back({s.P[{lev, bb}][l - 1], s.P[{lev, a}][l - 1], Sd + A->S_off[g], kb, ka, kl, kb, ka, kb, 0, 1, 1.0, 0.0});
        }
      // dense near blocks D_ts = F^l_t (F^l_s)^T, row-major = column-major F_s F_t^T
      double* Dd = A->st.D.as<double>();
      for (size_t q = 0; q < t->near.size(); ++q) {
        auto [a, bb] = t->near[q];
        const int ma = t->csize[cid(L, a)], mb = t->csize[cid(L, bb)];
        if (a == bb) {
          diag_cps.push_back({s.Ddiag[a].as<double>(), ma, Dd + A->D_off[q], ma, ma, ma, 1.0, 0.0, 0});
          continue;
        }
        const int l = sib_level(L, a, bb);
        const int kl = s.pair_rank(l, L, a);
        if (kl == 0) {  // an empty product (K = 0) writes the zero block, in the same launch
          gs.push_back({nullptr, nullptr, Dd + A->D_off[q], mb, ma, 0, 1, 1, mb, 0, 0, 1.0, 0.0});
          continue;
        }
        gs.push_back({s.Frows(l, L, bb), s.Frows(l, L, a), Dd + A->D_off[q], mb, ma, kl, n, n, mb, 0, 1, 1.0, 0.0});
      }
      s.J->out = std::move(A);
    }
    copy_batched(c, cps);
    copy_batched(c, diag_cps);
    gemm_batched(c, gs);
    H2_HIP(hipStreamSynchronize(c.s));
    c.scratch.clear();
    c.stage.reset();
  }
  const double t_recomp = now_ms() - t0;
  const double total = now_ms() - t_start;
  for (auto& s : js) {
    h2_build_stats& st = s.J->stats;
    for (int lev = 0; lev <= s.L; ++lev) {
      int mx = 0;
      for (int i = 0; i < (1 << lev); ++i) mx = std::max(mx, (int)s.rank[cid(lev, i)]);
      st.strong_rank[lev] = mx;
    }
    st.applies = s.S->applies - s.applies1;
    st.converged = s.J->converged;
    st.time_ms[0] = t_norm;
    st.time_ms[1] = t_sample;
    st.time_ms[2] = t_range;
    st.time_ms[3] = t_proj;
    st.time_ms[4] = t_diag;
    st.time_ms[5] = t_recomp;
    st.time_ms[7] = total;
  }
  if (verbose())
    std::fprintf(stderr, "  [h2_build] done: %zu problems, ms norm %.1f sample %.1f range %.1f proj %.1f diag %.1f recompress %.1f total %.1f\n",
                 jobs.size(), t_norm, t_sample, t_range, t_proj, t_diag, t_recomp, total);
}

std::unique_ptr<h2_matrix> build_h2(const h2_tree* t, Sampler& S, const BuildParams& prm, Ctx& c,
                                    h2_build_stats* st, bool* converged_out) {
  std::vector<BuildJob> jobs(1);
  jobs[0].t = t;
  jobs[0].S = &S;
  jobs[0].prm = prm;
  build_h2_multi(jobs, c);
  if (st) *st = jobs[0].stats;
  if (converged_out) *converged_out = jobs[0].converged;
  return std::move(jobs[0].out);
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

static BuildParams params_from(const h2_opts* opts) {
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
  return p;
}

h2_status h2_build_batched(int nprob, const h2_tree* const* trees, const h2_sampler_fn* samplers,
                           void* const* ctxs, const h2_opts* opts, hipStream_t stream,
                           h2_matrix** out, h2_build_stats* stats) {
  bool conv = true;
  h2_status st = guarded_status([&] {
    H2_CHECK(nprob >= 0 && (nprob == 0 || (trees && samplers && ctxs && opts && out)), H2_EINVAL,
             "null argument");
    for (int i = 0; i < nprob; ++i) {
      H2_CHECK(trees[i] && samplers[i], H2_EINVAL, "null tree or sampler");
      out[i] = nullptr;
    }
    std::vector<std::unique_ptr<UserSampler>> S;
    std::vector<BuildJob> jobs(nprob);
    for (int i = 0; i < nprob; ++i) {
      S.push_back(std::make_unique<UserSampler>(trees[i], samplers[i], ctxs[i]));
      jobs[i].t = trees[i];
      jobs[i].S = S.back().get();
      jobs[i].prm = params_from(&opts[i]);
    }
    Ctx c;
    c.s = stream;
    build_h2_multi(jobs, c);
    for (int i = 0; i < nprob; ++i) {
      if (stats) stats[i] = jobs[i].stats;
      conv = conv && jobs[i].converged;
      out[i] = jobs[i].out.release();
    }
  });
  if (st == H2_OK && !conv) return H2_ENOTCONVERGED;
  return st;
}

h2_status h2_build_batched_packed(int nprob, const h2_tree* const* trees,
                                  h2_batched_sampler_fn sampler, void* ctx, const h2_opts* opts,
                                  hipStream_t stream, h2_matrix** out, h2_build_stats* stats,
                                  int64_t* sampler_calls) {
  bool conv = true;
  h2_status st = guarded_status([&] {
    H2_CHECK(nprob >= 0 && (nprob == 0 || (trees && sampler && opts && out)), H2_EINVAL,
             "null argument");
    PackedBatch B;
    B.fn = sampler;
    B.ctx = ctx;
    B.off.assign(nprob + 1, 0);
    for (int i = 0; i < nprob; ++i) {
      H2_CHECK(trees[i], H2_EINVAL, "null tree");
      out[i] = nullptr;
      B.trees.push_back(trees[i]);
      B.off[i + 1] = B.off[i] + trees[i]->n;
    }
    std::vector<std::unique_ptr<PackedSampler>> S;
    std::vector<BuildJob> jobs(nprob);
    for (int i = 0; i < nprob; ++i) {
      S.push_back(std::make_unique<PackedSampler>(&B, i));
      jobs[i].t = trees[i];
      jobs[i].S = S.back().get();
      jobs[i].prm = params_from(&opts[i]);
    }
    Ctx c;
    c.s = stream;
    build_h2_multi(jobs, c);
    for (int i = 0; i < nprob; ++i) {
      if (stats) stats[i] = jobs[i].stats;
      conv = conv && jobs[i].converged;
      out[i] = jobs[i].out.release();
    }
    if (sampler_calls) *sampler_calls = B.calls;
  });
  if (st == H2_OK && !conv) return H2_ENOTCONVERGED;
  return st;
}

h2_status h2_build(const h2_tree* tree, h2_sampler_fn sampler, void* ctx, const h2_opts* opts,
                   hipStream_t stream, h2_matrix** out, h2_build_stats* stats) {
  bool conv = true;
  h2_status st = guarded_status([&] {
    H2_CHECK(tree && sampler && opts && out, H2_EINVAL, "null argument");
    BuildParams p = params_from(opts);
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
