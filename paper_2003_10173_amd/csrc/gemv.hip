// H2 matrix storage and HGEMV (Sec. 3.2: the four-stage product
// A x = D x + U (S (V^T x)) -- upsweep through the basis tree, coupling
// products at every level, downsweep, and the block-sparse dense product).
//
// Device layout (level-ordered, tree-order rows):
//   U  per leaf i: |leaf| x k row-major, leaves concatenated
//   E  per non-root cluster c: k_c x k_parent row-major
//   S  per far pair (CSR by row cluster, levels ascending): k_t x k_s row-major
//   D  per near pair (CSR by row leaf): |t| x |s| row-major
//   coefficient vectors x^, y^: per cluster k_c x nv column-major, clusters
//   concatenated in global order (offset kpre[c] * nv)
//   multivectors: tree order, column-major (ld >= n)
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "kernels_common.h"

namespace h2 {

// ------------------------------------------------------------------ layout
void matrix_layout(h2_matrix* A, const h2_tree* t, const std::vector<int32_t>& rank) {
  const int L = t->L, ncl = t->nclusters();
  H2_CHECK((int)rank.size() == ncl, H2_EINVAL, "rank array size mismatch");
  A->tree = t;
  A->rank = rank;
  A->rank[0] = 0;  // the root has no far field
  A->U_off.assign((1 << L) + 1, 0);
  for (int i = 0; i < (1 << L); ++i)
    A->U_off[i + 1] = A->U_off[i] + (int64_t)t->csize[cid(L, i)] * A->rank[cid(L, i)];
  A->E_off.assign(ncl + 1, 0);
  for (int c = 0; c < ncl; ++c) {
    int64_t sz = 0;
    if (c > 0) sz = (int64_t)A->rank[c] * A->rank[(c - 1) / 2];
    A->E_off[c + 1] = A->E_off[c] + sz;
  }
  const int64_t nfar = t->num_far();
  A->S_off.assign(nfar + 1, 0);
  for (int l = 1; l <= L; ++l)
    for (int64_t g = t->far_base[l]; g < t->far_base[l + 1]; ++g) {
      int a = t->far[l][g - t->far_base[l]].first, b = t->far[l][g - t->far_base[l]].second;
      A->S_off[g + 1] = (int64_t)A->rank[cid(l, a)] * A->rank[cid(l, b)];
    }
  for (int64_t g = 0; g < nfar; ++g) A->S_off[g + 1] += A->S_off[g];
  const int64_t nnear = (int64_t)t->near.size();
  A->D_off.assign(nnear + 1, 0);
  for (int64_t g = 0; g < nnear; ++g)
    A->D_off[g + 1] = A->D_off[g] + (int64_t)t->csize[cid(L, t->near[g].first)] *
                                        t->csize[cid(L, t->near[g].second)];
  A->kpre.assign(ncl + 1, 0);
  A->kmax = 0;
  for (int c = 0; c < ncl; ++c) {
    A->kpre[c + 1] = A->kpre[c] + A->rank[c];
    A->kmax = std::max(A->kmax, (int)A->rank[c]);
  }
  tree_device(t);
  upload(A->d_rank, A->rank);
  upload(A->d_U_off, A->U_off);
  upload(A->d_E_off, A->E_off);
  upload(A->d_S_off, A->S_off);
  upload(A->d_D_off, A->D_off);
  upload(A->d_kpre, A->kpre);
}

void matrix_alloc(h2_matrix* A, h2_precision prec) {
  A->st.prec = prec;
  const size_t e = A->st.elem();
  A->st.U.alloc(std::max<int64_t>(A->nU(), 1) * e);
  A->st.E.alloc(std::max<int64_t>(A->nE(), 1) * e);
  A->st.S.alloc(std::max<int64_t>(A->nS(), 1) * e);
  A->st.D.alloc(std::max<int64_t>(A->nD(), 1) * e);
}

std::unique_ptr<h2_matrix> matrix_clone_layout(const h2_matrix* A) {
  auto B = std::make_unique<h2_matrix>();
  matrix_layout(B.get(), A->tree, A->rank);
  return B;
}

// ------------------------------------------------------------------ kernels
template <class M, class V>
__global__ void k_up_leaf(int L, const int32_t* __restrict__ cstart,
                          const int32_t* __restrict__ csize, const int32_t* __restrict__ rank,
                          const int64_t* __restrict__ kpre, const int64_t* __restrict__ Uoff,
                          const M* __restrict__ U, const V* __restrict__ x, int ldx, int nv,
                          V* __restrict__ xh) {
  const int i = blockIdx.x;
  const int c = (1 << L) - 1 + i;
  const int k = rank[c];
  if (k == 0) return;
  const int r0 = cstart[c], m = csize[c];
  const M* Ui = U + Uoff[i];
  V* out = xh + kpre[c] * nv;
  for (int idx = threadIdx.x; idx < k * nv; idx += blockDim.x) {
    const int j = idx % k, v = idx / k;
    const V* xv = x + (size_t)v * ldx + r0;
    V s = 0;
    for (int r = 0; r < m; ++r) s += to_acc<V>(Ui[(size_t)r * k + j]) * xv[r];
    out[(size_t)v * k + j] = s;
  }
}

template <class M, class V>
__global__ void k_up_transfer(int l, const int32_t* __restrict__ rank,
                              const int64_t* __restrict__ kpre, const int64_t* __restrict__ Eoff,
                              const M* __restrict__ E, int nv, V* __restrict__ xh) {
  const int p = blockIdx.x;
  const int cp = (1 << l) - 1 + p;
  const int kp = rank[cp];
  if (kp == 0) return;
  const int c1 = (1 << (l + 1)) - 1 + 2 * p, c2 = c1 + 1;
  const int k1 = rank[c1], k2 = rank[c2];
  const M* E1 = E + Eoff[c1];
  const M* E2 = E + Eoff[c2];
  for (int idx = threadIdx.x; idx < kp * nv; idx += blockDim.x) {
    const int j = idx % kp, v = idx / kp;
    const V* x1 = xh + kpre[c1] * nv + (size_t)v * k1;
    const V* x2 = xh + kpre[c2] * nv + (size_t)v * k2;
    V s = 0;
    for (int q = 0; q < k1; ++q) s += to_acc<V>(E1[(size_t)q * kp + j]) * x1[q];
    for (int q = 0; q < k2; ++q) s += to_acc<V>(E2[(size_t)q * kp + j]) * x2[q];
    xh[kpre[cp] * nv + (size_t)v * kp + j] = s;
  }
}

// one block per non-root cluster (all levels in one launch)
template <class M, class V>
__global__ void k_coupling(const int32_t* __restrict__ rank, const int64_t* __restrict__ kpre,
                           const int32_t* __restrict__ far_ptr,
                           const int32_t* __restrict__ far_col, const int64_t* __restrict__ Soff,
                           const M* __restrict__ S, int nv, const V* __restrict__ xh,
                           V* __restrict__ yh) {
  const int c = blockIdx.x + 1;
  const int kt = rank[c];
  if (kt == 0) return;
  int l = 31 - __clz(c + 1);
  const int base = (1 << l) - 1;
  const int pb = far_ptr[c + l], pe = far_ptr[c + l + 1];
  V* out = yh + kpre[c] * nv;
  for (int idx = threadIdx.x; idx < kt * nv; idx += blockDim.x) {
    const int j = idx % kt, v = idx / kt;
    V s = 0;
    for (int g = pb; g < pe; ++g) {
      const int cs = base + far_col[g];
      const int ks = rank[cs];
      const M* Sg = S + Soff[g] + (size_t)j * ks;
      const V* xs = xh + kpre[cs] * nv + (size_t)v * ks;
      for (int q = 0; q < ks; ++q) s += to_acc<V>(Sg[q]) * xs[q];
    }
    out[(size_t)v * kt + j] = s;
  }
}

template <class M, class V>
__global__ void k_down_transfer(int l, const int32_t* __restrict__ rank,
                                const int64_t* __restrict__ kpre,
                                const int64_t* __restrict__ Eoff, const M* __restrict__ E, int nv,
                                V* __restrict__ yh) {
  const int ch = blockIdx.x;
  const int cc = (1 << l) - 1 + ch;
  const int cp = (1 << (l - 1)) - 1 + ch / 2;
  const int kc = rank[cc], kp = rank[cp];
  if (kc == 0 || kp == 0) return;
  const M* Ec = E + Eoff[cc];
  for (int idx = threadIdx.x; idx < kc * nv; idx += blockDim.x) {
    const int j = idx % kc, v = idx / kc;
    const V* yp = yh + kpre[cp] * nv + (size_t)v * kp;
    V s = 0;
    for (int q = 0; q < kp; ++q) s += to_acc<V>(Ec[(size_t)j * kp + q]) * yp[q];
    yh[kpre[cc] * nv + (size_t)v * kc + j] += s;
  }
}

// y_leaf = alpha (U y^ + sum_near D x_s) + beta y_leaf; one block per (leaf, 32 columns)
constexpr int LEAF_MAX = 64;
constexpr int NVC = 32;

template <class M, class V>
__global__ __launch_bounds__(256) void k_leaf_out(
    int L, const int32_t* __restrict__ cstart, const int32_t* __restrict__ csize,
    const int32_t* __restrict__ rank, const int64_t* __restrict__ kpre,
    const int64_t* __restrict__ Uoff, const M* __restrict__ U,
    const int32_t* __restrict__ near_ptr, const int32_t* __restrict__ near_col,
    const int64_t* __restrict__ Doff, const M* __restrict__ D, int nv, const V* __restrict__ yh,
    const V* __restrict__ x, int ldx, V alpha, V beta, V* __restrict__ y, int ldy) {
  __shared__ V Ds[LEAF_MAX * LEAF_MAX];
  __shared__ V xs[LEAF_MAX * NVC];
  const int i = blockIdx.x;
  const int c = (1 << L) - 1 + i;
  const int r0 = cstart[c], m = csize[c];
  const int v0 = blockIdx.y * NVC;
  const int nvc = min(NVC, nv - v0);
  const int tid = threadIdx.x;
  constexpr int PER = LEAF_MAX * NVC / 256;
  V acc[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) acc[q] = 0;
  const int leaf_base = (1 << L) - 1;
  for (int g = near_ptr[i]; g < near_ptr[i + 1]; ++g) {
    const int s = near_col[g];
    const int s0 = cstart[leaf_base + s], ms = csize[leaf_base + s];
    const M* Dg = D + Doff[g];
    for (int e = tid; e < m * ms; e += 256) Ds[e] = to_acc<V>(Dg[e]);
    for (int e = tid; e < ms * NVC; e += 256) {
      const int cc = e / NVC, v = e % NVC;
      xs[e] = v < nvc ? x[(size_t)(v0 + v) * ldx + s0 + cc] : V(0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / NVC, v = idx % NVC;
      if (r < m) {
        V s_ = 0;
        for (int cc = 0; cc < ms; ++cc) s_ += Ds[r * ms + cc] * xs[cc * NVC + v];
        acc[q] += s_;
      }
    }
    __syncthreads();
  }
  const int k = rank[c];
  const M* Ui = U + Uoff[i];
  const V* yhi = yh + kpre[c] * nv;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + 256 * q;
    const int r = idx / NVC, v = idx % NVC;
    if (r < m && v < nvc) {
      V s_ = acc[q];
      for (int j = 0; j < k; ++j) s_ += to_acc<V>(Ui[(size_t)r * k + j]) * yhi[(size_t)(v0 + v) * k + j];
      V* yp = y + (size_t)(v0 + v) * ldy + r0 + r;
      *yp = beta == V(0) ? alpha * s_ : alpha * s_ + beta * *yp;
    }
  }
}

template <class V>
__global__ void k_gather(int n, int nv, const int32_t* __restrict__ perm, const V* __restrict__ x,
                         int ldx, V* __restrict__ xt, int ldt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * nv) return;
  const int r = (int)(e % n), v = (int)(e / n);
  xt[(size_t)v * ldt + r] = x[(size_t)v * ldx + perm[r]];
}

template <class V>
__global__ void k_scatter(int n, int nv, const int32_t* __restrict__ perm, V alpha,
                          const V* __restrict__ yt, int ldt, V beta, V* __restrict__ y, int ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * nv) return;
  const int r = (int)(e % n), v = (int)(e / n);
  V* yp = y + (size_t)v * ldy + perm[r];
  const V val = alpha * yt[(size_t)v * ldt + r];
  *yp = beta == V(0) ? val : val + beta * *yp;
}

// ------------------------------------------------------------------ drivers
template <class M, class V>
static void gemv_tree_impl(const h2_matrix* A, int nv, V alpha, const V* xt, int ldx, V beta,
                           V* yt, int ldy, hipStream_t s) {
  const h2_tree* t = A->tree;
  const int L = t->L;
  const int64_t ktot = A->kpre.back();
  const size_t need = (size_t)2 * ktot * nv * sizeof(V);
  A->ws.reserve(std::max<size_t>(need, 256));
  V* xh = A->ws.as<V>();
  V* yh = xh + ktot * nv;
  const M* U = A->st.U.as<M>();
  const M* E = A->st.E.as<M>();
  const M* S = A->st.S.as<M>();
  const M* D = A->st.D.as<M>();
  const int32_t* rank = A->d_rank.as<int32_t>();
  const int64_t* kpre = A->d_kpre.as<int64_t>();
  if (ktot > 0 && L >= 1) {
    k_up_leaf<M, V><<<1 << L, 256, 0, s>>>(L, t->d_cstart.as<int32_t>(), t->d_csize.as<int32_t>(),
                                            rank, kpre, A->d_U_off.as<int64_t>(), U, xt, ldx, nv,
                                            xh);
    for (int l = L - 1; l >= 1; --l)
      k_up_transfer<M, V><<<1 << l, 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv,
                                                  xh);
    k_coupling<M, V><<<t->nclusters() - 1, 256, 0, s>>>(
        rank, kpre, t->d_far_ptr.as<int32_t>(), t->d_far_col.as<int32_t>(),
        A->d_S_off.as<int64_t>(), S, nv, xh, yh);
    for (int l = 2; l <= L; ++l)
      k_down_transfer<M, V><<<1 << l, 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv,
                                                    yh);
  }
  dim3 grid(1 << L, (nv + NVC - 1) / NVC);
  k_leaf_out<M, V><<<grid, 256, 0, s>>>(
      L, t->d_cstart.as<int32_t>(), t->d_csize.as<int32_t>(), rank, kpre,
      A->d_U_off.as<int64_t>(), U, t->d_near_ptr.as<int32_t>(), t->d_near_col.as<int32_t>(),
      A->d_D_off.as<int64_t>(), D, nv, yh, xt, ldx, alpha, beta, yt, ldy);
  H2_LAUNCH_CHECK();
}

void gemv_tree_f64(const h2_matrix* A, int nv, double alpha, const double* xt, int ldx,
                   double beta, double* yt, int ldy, hipStream_t s) {
  if (nv <= 0) return;
  H2_CHECK(A->st.prec == H2_FP64, H2_EINVAL, "FP64 HGEMV needs an FP64 matrix");
  gemv_tree_impl<double, double>(A, nv, alpha, xt, ldx, beta, yt, ldy, s);
}

void gemv_tree_f32(const h2_matrix* A, int nv, float alpha, const float* xt, int ldx, float beta,
                   float* yt, int ldy, hipStream_t s) {
  if (nv <= 0) return;
  switch (A->st.prec) {
    case H2_FP64: gemv_tree_impl<double, float>(A, nv, alpha, xt, ldx, beta, yt, ldy, s); break;
    case H2_FP32: gemv_tree_impl<float, float>(A, nv, alpha, xt, ldx, beta, yt, ldy, s); break;
    case H2_BF16: gemv_tree_impl<bf16_t, float>(A, nv, alpha, xt, ldx, beta, yt, ldy, s); break;
  }
}

void gather_rows(const h2_tree* t, int nv, const double* x, int ldx, double* xt, int ldt,
                 hipStream_t s) {
  const int64_t tot = (int64_t)t->n * nv;
  if (tot == 0) return;
  k_gather<double><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(t->n, nv, t->d_perm.as<int32_t>(),
                                                                 x, ldx, xt, ldt);
  H2_LAUNCH_CHECK();
}
void scatter_rows(const h2_tree* t, int nv, double alpha, const double* yt, int ldt, double beta,
                  double* y, int ldy, hipStream_t s) {
  const int64_t tot = (int64_t)t->n * nv;
  if (tot == 0) return;
  k_scatter<double><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(
      t->n, nv, t->d_perm.as<int32_t>(), alpha, yt, ldt, beta, y, ldy);
  H2_LAUNCH_CHECK();
}
void gather_rows_f32(const h2_tree* t, int nv, const float* x, int ldx, float* xt, int ldt,
                     hipStream_t s) {
  const int64_t tot = (int64_t)t->n * nv;
  if (tot == 0) return;
  k_gather<float><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(t->n, nv, t->d_perm.as<int32_t>(),
                                                                x, ldx, xt, ldt);
  H2_LAUNCH_CHECK();
}
void scatter_rows_f32(const h2_tree* t, int nv, float alpha, const float* yt, int ldt, float beta,
                      float* y, int ldy, hipStream_t s) {
  const int64_t tot = (int64_t)t->n * nv;
  if (tot == 0) return;
  k_scatter<float><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(
      t->n, nv, t->d_perm.as<int32_t>(), alpha, yt, ldt, beta, y, ldy);
  H2_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ conversions
template <class Src, class Dst>
__global__ void k_convert(int64_t n, const Src* __restrict__ a, Dst* __restrict__ b, double scale) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = from_double<Dst>(to_double(a[e]) * scale);
}

template <class Src, class Dst>
static void convert_buf(int64_t n, const void* a, void* b, double scale, hipStream_t s) {
  if (n <= 0) return;
  k_convert<Src, Dst><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, (const Src*)a, (Dst*)b, scale);
  H2_LAUNCH_CHECK();
}

// copy storage of A into B (same layout) converting precision and scaling S, D
void matrix_copy_convert(const h2_matrix* A, h2_matrix* B, double scale, hipStream_t s) {
  auto run = [&](int64_t n, const DevBuf& a, DevBuf& b, double sc) {
    if (A->st.prec == H2_FP64) {
      if (B->st.prec == H2_FP64) convert_buf<double, double>(n, a.p, b.p, sc, s);
      else if (B->st.prec == H2_FP32) convert_buf<double, float>(n, a.p, b.p, sc, s);
      else convert_buf<double, bf16_t>(n, a.p, b.p, sc, s);
    } else if (A->st.prec == H2_FP32) {
      if (B->st.prec == H2_FP64) convert_buf<float, double>(n, a.p, b.p, sc, s);
      else if (B->st.prec == H2_FP32) convert_buf<float, float>(n, a.p, b.p, sc, s);
      else convert_buf<float, bf16_t>(n, a.p, b.p, sc, s);
    } else {
      if (B->st.prec == H2_FP64) convert_buf<bf16_t, double>(n, a.p, b.p, sc, s);
      else if (B->st.prec == H2_FP32) convert_buf<bf16_t, float>(n, a.p, b.p, sc, s);
      else convert_buf<bf16_t, bf16_t>(n, a.p, b.p, sc, s);
    }
  };
  run(A->nU(), A->st.U, B->st.U, 1.0);
  run(A->nE(), A->st.E, B->st.E, 1.0);
  run(A->nS(), A->st.S, B->st.S, scale);
  run(A->nD(), A->st.D, B->st.D, scale);
}

__global__ void k_identity_blocks(int L, const int32_t* __restrict__ csize,
                                  const int32_t* __restrict__ near_ptr,
                                  const int32_t* __restrict__ near_col,
                                  const int64_t* __restrict__ Doff, double alpha,
                                  double* __restrict__ D) {
  const int i = blockIdx.x;
  const int m = csize[(1 << L) - 1 + i];
  for (int g = near_ptr[i]; g < near_ptr[i + 1]; ++g) {
    const int s = near_col[g];
    const int ms = csize[(1 << L) - 1 + s];
    double* Dg = D + Doff[g];
    for (int e = threadIdx.x; e < m * ms; e += blockDim.x)
      Dg[e] = (s == i && e / ms == e % ms) ? alpha : 0.0;
  }
}

void matrix_identity(h2_matrix* A, const h2_tree* t, double alpha, hipStream_t s) {
  std::vector<int32_t> rank(t->nclusters(), 0);
  matrix_layout(A, t, rank);
  matrix_alloc(A, H2_FP64);
  k_identity_blocks<<<1 << t->L, 256, 0, s>>>(t->L, t->d_csize.as<int32_t>(),
                                               t->d_near_ptr.as<int32_t>(),
                                               t->d_near_col.as<int32_t>(),
                                               A->d_D_off.as<int64_t>(), alpha,
                                               A->st.D.as<double>());
  H2_LAUNCH_CHECK();
}

}  // namespace h2
