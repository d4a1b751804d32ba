// Test hooks (include/h2_testing.h): host-array wrappers around the batched
// primitives and access to the weak factors of the last kept build.
#include <functional>
#include <vector>

#include "h2_testing.h"
#include "internal.h"
#include "linalg.h"

namespace h2 {
h2_status guarded_status(const std::function<void()>& f);

thread_local bool g_keep_factors = false;
thread_local std::vector<std::vector<int32_t>> g_factor_ranks;
thread_local std::vector<std::vector<double>> g_factor_F;
thread_local std::vector<int> g_factor_K;

void keep_factors(int l, const std::vector<int>& k, int K, const double* F_dev, int n) {
  if (!g_keep_factors) return;
  if ((int)g_factor_F.size() <= l) {
    g_factor_F.resize(l + 1);
    g_factor_ranks.resize(l + 1);
    g_factor_K.resize(l + 1, 0);
  }
  g_factor_ranks[l].assign(k.begin(), k.end());
  g_factor_K[l] = K;
  g_factor_F[l].assign((size_t)n * K, 0.0);
  if (K > 0) H2_HIP(hipMemcpy(g_factor_F[l].data(), F_dev, (size_t)n * K * sizeof(double), hipMemcpyDeviceToHost));
}
void reset_factors() {
  if (!g_keep_factors) return;
  g_factor_F.clear();
  g_factor_ranks.clear();
  g_factor_K.clear();
}
}  // namespace h2

using namespace h2;

extern "C" {

h2_status h2_test_gemm(int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
                       const double* B, int ldb, double beta, double* C, int ldc) {
  return guarded_status([&] {
    const size_t na = (size_t)lda * (ta ? M : K), nb = (size_t)ldb * (tb ? K : N), nc = (size_t)ldc * N;
    DevBuf a(na * 8 + 8), b(nb * 8 + 8), c(nc * 8 + 8);
    H2_HIP(hipMemcpy(a.p, A, na * 8, hipMemcpyHostToDevice));
    H2_HIP(hipMemcpy(b.p, B, nb * 8, hipMemcpyHostToDevice));
    H2_HIP(hipMemcpy(c.p, C, nc * 8, hipMemcpyHostToDevice));
    Ctx ctx;
    std::vector<GemmDesc> d{{a.as<double>(), b.as<double>(), c.as<double>(), M, N, K, lda, ldb, ldc, ta, tb, alpha, beta}};
    gemm_batched(ctx, d);
    H2_HIP(hipDeviceSynchronize());
    H2_HIP(hipMemcpy(C, c.p, nc * 8, hipMemcpyDeviceToHost));
  });
}

h2_status h2_test_qr(int m, int n, const double* A, double* Q, double* R) {
  return guarded_status([&] {
    const int k = std::min(m, n);
    DevBuf a((size_t)m * n * 8), q((size_t)m * k * 8 + 8), r((size_t)k * n * 8 + 8);
    H2_HIP(hipMemcpy(a.p, A, (size_t)m * n * 8, hipMemcpyHostToDevice));
    Ctx ctx;
    std::vector<QRDesc> d{{a.as<double>(), m, m, n, Q ? q.as<double>() : nullptr, m, R ? r.as<double>() : nullptr, k}};
    qr_batched(ctx, d);
    H2_HIP(hipDeviceSynchronize());
    if (Q) H2_HIP(hipMemcpy(Q, q.p, (size_t)m * k * 8, hipMemcpyDeviceToHost));
    if (R) H2_HIP(hipMemcpy(R, r.p, (size_t)k * n * 8, hipMemcpyDeviceToHost));
  });
}

h2_status h2_test_cholqr(int m, int n, const double* A, double* Q, double* R, int mode) {
  return guarded_status([&] {
    H2_CHECK(mode >= 0 && mode <= 3, H2_EINVAL, "mode must be 0..3");
    DevBuf a((size_t)m * n * 8), r((size_t)n * n * 8);
    H2_HIP(hipMemcpy(a.p, A, (size_t)m * n * 8, hipMemcpyHostToDevice));
    H2_HIP(hipMemset(r.p, 0, (size_t)n * n * 8));
    Ctx ctx;
    std::vector<CholQRDesc> d{{a.as<double>(), m, m, n, r.as<double>(), n}};
    if (mode == 1) {
      qr_blocked(ctx, d);
    } else if (mode >= 2) {
      DevBuf q((size_t)m * n * 8);
      std::vector<QRDesc> t{{a.as<double>(), m, m, n, mode == 2 ? q.as<double>() : nullptr, m,
                             r.as<double>(), n}};
      qr_auto(ctx, t);
      H2_HIP(hipDeviceSynchronize());
      if (mode == 2) H2_HIP(hipMemcpy(a.p, q.p, (size_t)m * n * 8, hipMemcpyDeviceToDevice));
    } else {
      DevBuf q((size_t)m * n * 8);
      std::vector<QRDesc> t{{a.as<double>(), m, m, n, q.as<double>(), m, r.as<double>(), n}};
      qr_tall_batched(ctx, t);
      H2_HIP(hipDeviceSynchronize());
      H2_HIP(hipMemcpy(a.p, q.p, (size_t)m * n * 8, hipMemcpyDeviceToDevice));
    }
    H2_HIP(hipDeviceSynchronize());
    if (Q) H2_HIP(hipMemcpy(Q, a.p, (size_t)m * n * 8, hipMemcpyDeviceToHost));
    if (R) H2_HIP(hipMemcpy(R, r.p, (size_t)n * n * 8, hipMemcpyDeviceToHost));
  });
}

h2_status h2_test_svd(int m, int n, const double* A, double* sigma, double* U, double* V) {
  return guarded_status([&] {
    DevBuf a((size_t)m * n * 8), s((size_t)n * 8), u((size_t)m * n * 8), v((size_t)n * n * 8);
    H2_HIP(hipMemcpy(a.p, A, (size_t)m * n * 8, hipMemcpyHostToDevice));
    Ctx ctx;
    std::vector<SVDDesc> d{{a.as<double>(), m, m, n, s.as<double>(), U ? u.as<double>() : nullptr, m, V ? v.as<double>() : nullptr, n}};
    svd_batched(ctx, d);
    H2_HIP(hipDeviceSynchronize());
    H2_HIP(hipMemcpy(sigma, s.p, (size_t)n * 8, hipMemcpyDeviceToHost));
    if (U) H2_HIP(hipMemcpy(U, u.p, (size_t)m * n * 8, hipMemcpyDeviceToHost));
    if (V) H2_HIP(hipMemcpy(V, v.p, (size_t)n * n * 8, hipMemcpyDeviceToHost));
  });
}

h2_status h2_test_svd_batch(int count, const int* m, const int* n, const double* A, double* sigma,
                            double* U, double* V) {
  return guarded_status([&] {
    H2_CHECK(count >= 0 && m && n && A && sigma && U && V, H2_EINVAL, "null argument");
    size_t na = 0, ns = 0, nv = 0;
    for (int i = 0; i < count; ++i) {
      H2_CHECK(m[i] >= n[i] && n[i] >= 0, H2_EINVAL, "needs m >= n >= 0");
      na += (size_t)m[i] * n[i];
      ns += n[i];
      nv += (size_t)n[i] * n[i];
    }
    DevBuf a(na * 8 + 8), s(ns * 8 + 8), u(na * 8 + 8), v(nv * 8 + 8);
    H2_HIP(hipMemcpy(a.p, A, na * 8, hipMemcpyHostToDevice));
    std::vector<SVDDesc> d;
    size_t oa = 0, os = 0, ov = 0;
    for (int i = 0; i < count; ++i) {
      d.push_back({a.as<double>() + oa, m[i], m[i], n[i], s.as<double>() + os, u.as<double>() + oa,
                   m[i], v.as<double>() + ov, n[i]});
      oa += (size_t)m[i] * n[i];
      os += n[i];
      ov += (size_t)n[i] * n[i];
    }
    Ctx ctx;
    svd_batched(ctx, d);
    H2_HIP(hipDeviceSynchronize());
    H2_HIP(hipMemcpy(sigma, s.p, ns * 8, hipMemcpyDeviceToHost));
    H2_HIP(hipMemcpy(U, u.p, na * 8, hipMemcpyDeviceToHost));
    H2_HIP(hipMemcpy(V, v.p, nv * 8, hipMemcpyDeviceToHost));
  });
}

void h2_test_keep_factors(int on) { g_keep_factors = on != 0; }

h2_status h2_test_factors(int level, int32_t* ranks_out, int* K_out, double* F_out) {
  return guarded_status([&] {
    H2_CHECK(level >= 1 && level < (int)g_factor_F.size(), H2_EINVAL, "no kept factors for level");
    if (ranks_out) std::copy(g_factor_ranks[level].begin(), g_factor_ranks[level].end(), ranks_out);
    if (K_out) *K_out = g_factor_K[level];
    if (F_out) std::copy(g_factor_F[level].begin(), g_factor_F[level].end(), F_out);
  });
}

}  // extern "C"
