// Test hooks (include/h2_testing.h): host-array wrappers around the batched
// primitives and access to the weak factors of the last kept build.
#include <functional>
#include <vector>

#include "h2_testing.h"
#include "internal.h"
#include "kernels_common.h"
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
// one 16x16 MFMA per kind (0: f64 16x16x4, 1: f32 16x16x4, 2: bf16 16x16x16)
// with A[i][0] = i + 1, A[i][1] = 1, B[0][j] = 1, B[1][j] = 32 (j + 1) (exact in
// bf16), every
// other k zero, operands placed as A[i][k] in lane i + 16 (k / kpl), element
// k % kpl, and B[k][j] in lane j + 16 (k / kpl), element k % kpl (kpl = k
// values per lane); out[lane * 4 + reg] = raw accumulator register.
typedef double t_d4 __attribute__((ext_vector_type(4)));
typedef float t_f4 __attribute__((ext_vector_type(4)));
typedef short t_s4 __attribute__((ext_vector_type(4)));
__global__ void k_mfma_probe(int kind, double* out) {
  const int l = threadIdx.x, i = l & 15, kg = l >> 4;
  auto aval = [&](int k) { return k == 0 ? (double)(i + 1) : (k == 1 ? 1.0 : 0.0); };
  auto bval = [&](int k) { return k == 0 ? 1.0 : (k == 1 ? 32.0 * (i + 1) : 0.0); };
  if (kind == 0) {
    t_d4 c = {0, 0, 0, 0};
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(aval(kg), bval(kg), c, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = c[r];
  } else if (kind == 1) {
    t_f4 c = {0, 0, 0, 0};
    c = __builtin_amdgcn_mfma_f32_16x16x4f32((float)aval(kg), (float)bval(kg), c, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = c[r];
  } else {
    t_s4 a, b;
    for (int e = 0; e < 4; ++e) {
      a[e] = (short)float_to_bf16((float)aval(4 * kg + e)).bits;
      b[e] = (short)float_to_bf16((float)bval(4 * kg + e)).bits;
    }
    t_f4 c = {0, 0, 0, 0};
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = c[r];
  }
}

// every lane's value of the double wave sum of in[0..63]
__global__ void k_wave_sum_probe(const double* __restrict__ in, double* __restrict__ out) {
  out[threadIdx.x] = wave_sum(in[threadIdx.x]);
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

void h2_test_svd_spin_limit(int polls) { svd_spin_limit = polls < 0 ? 0 : polls; }

h2_status h2_test_mfma_layout(int kind, double* out) {
  return guarded_status([&] {
    H2_CHECK(kind >= 0 && kind <= 2 && out, H2_EINVAL, "kind 0..2 and out needed");
    DevBuf o(256 * 8);
    k_mfma_probe<<<1, 64>>>(kind, o.as<double>());
    H2_LAUNCH_CHECK();
    H2_HIP(hipDeviceSynchronize());
    H2_HIP(hipMemcpy(out, o.p, 256 * 8, hipMemcpyDeviceToHost));
  });
}

h2_status h2_test_wave_sum(const double* in, double* out) {
  return guarded_status([&] {
    H2_CHECK(in && out, H2_EINVAL, "in and out needed");
    DevBuf b(128 * 8);
    H2_HIP(hipMemcpy(b.p, in, 64 * 8, hipMemcpyHostToDevice));
    k_wave_sum_probe<<<1, 64>>>(b.as<double>(), b.as<double>() + 64);
    H2_LAUNCH_CHECK();
    H2_HIP(hipDeviceSynchronize());
    H2_HIP(hipMemcpy(out, b.as<double>() + 64, 64 * 8, hipMemcpyDeviceToHost));
  });
}

h2_status h2_test_gemv_tile(const h2_matrix* A, int nv, const double* x, double* y, int nt) {
  return guarded_status([&] {
    H2_CHECK(A && x && y && nv > 0 && A->st.prec == H2_FP64, H2_EINVAL, "bad arguments");
    const int n = A->tree->n;
    DevBuf w((size_t)2 * n * nv * sizeof(double));
    double* xt = w.as<double>();
    double* yt = xt + (size_t)n * nv;
    gather_rows(A->tree, nv, x, n, xt, n, 0);
    gemv_tree_f64(A, nv, 1.0, xt, n, 0.0, yt, n, 0, nt);
    scatter_rows(A->tree, nv, 1.0, yt, n, 0.0, y, n, 0);
    H2_HIP(hipDeviceSynchronize());
  });
}

int h2_test_tuned_tile(const h2_matrix* A, int nv) {
  if (!A) return -1;
  auto it = A->tree->tuned_nt.find(std::tuple<int, int, int>{std::min((nv + 15) / 16, 4), 8, 8});
  return it == A->tree->tuned_nt.end() ? 0 : it->second;
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
