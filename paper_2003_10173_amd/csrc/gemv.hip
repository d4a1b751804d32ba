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
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <type_traits>

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
// Workgroups are dealt to the 8 XCDs in turn (workgroup b runs on XCD
// b mod 8, each XCD with its own L2).  xcd_local maps them so that every XCD
// takes a contiguous range of [0, n): tree-ordered leaves are spatially
// close, so the multivector blocks that neighbouring leaves share stay in
// one L2.  The identity when n is not a multiple of 8.
__device__ inline int xcd_local(int b, int n) {
  constexpr int NX = 8;
  if (n % NX) return b;
  return (b % NX) * (n / NX) + b / NX;
}

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

// Matrix-core version of the leaf stage for FP64 x FP64, FP32 x FP32 and
// BF16 x FP32 (BF16 operands, FP32 accumulation): y_leaf = alpha (U_t y^_t +
// sum_near D_ts x_s) + beta y_leaf as a block-sparse product.  One workgroup
// per (leaf, 16*NT vectors); wave w owns rows 16w..16w+15 and NT 16x16 output
// tiles.  Each source block (a near D_ts with x_s, or U_t with y^_t) is staged
// in LDS with coalesced loads (A row-major, zero-padded in k), then consumed
// by 16x16xK MFMAs: K = 4 for f64 and f32, 16 for bf16.
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef short mf_s4 __attribute__((ext_vector_type(4)));

template <class M> struct MfmaTraits;
template <> struct MfmaTraits<double> {
  using SA = double; using SB = double; using Acc = mf_d4;
  static constexpr int KS = 4, ALD = 64 + 2, PADB = 2;
};
template <> struct MfmaTraits<float> {
  using SA = float; using SB = float; using Acc = mf_f4;
  static constexpr int KS = 4, ALD = 64 + 4, PADB = 4;
};
template <> struct MfmaTraits<bf16_t> {
  using SA = uint16_t; using SB = uint16_t; using Acc = mf_f4;
  static constexpr int KS = 16, ALD = 64 + 8, PADB = 8;
};

__device__ inline double mf_a(double x) { return x; }
__device__ inline float mf_a(float x) { return x; }
__device__ inline uint16_t mf_a(bf16_t x) { return x.bits; }
template <class SB, class V> __device__ inline SB mf_b(V x);
template <> __device__ inline double mf_b<double, double>(double x) { return x; }
template <> __device__ inline float mf_b<float, float>(float x) { return x; }
template <> __device__ inline uint16_t mf_b<uint16_t, float>(float x) { return float_to_bf16(x).bits; }

// Block-row product on matrix cores: out (rows x nvc) = sum over sources q of
// A_q (rows x K_q) B_q (K_q x nvc); A_q row-major (or, transA, the transpose
// of a row-major K_q x rows block), B_q column-major with leading dimension
// ldb_q.  The workgroup's 4 waves own 16 rows each (rows <= 64), NT 16-column
// output tiles each; the result stays in acc (register layout as described
// at the epilogues).
template <class M, class V, int NT, class Src>
__device__ inline void blockrow_mfma(int rows, int nsrc, const Src& src, int nvc,
                                     typename MfmaTraits<M>::Acc (&acc)[NT],
                                     typename MfmaTraits<M>::SA* As,
                                     typename MfmaTraits<M>::SB* Bs) {
  using T = MfmaTraits<M>;
  using SA = typename T::SA;
  using SB = typename T::SB;
  constexpr bool BF = T::KS == 16;
  constexpr int NC = 16 * NT;
  constexpr int ALD = T::ALD;
  constexpr int BLD = BF ? 64 + T::PADB : NC + T::PADB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[ct][r] = 0;
  for (int q = 0; q < nsrc; ++q) {
    const M* Ap;
    const V* Bp;
    int K, ldb;
    bool transA;
    src(q, Ap, K, transA, Bp, ldb);
    if (K == 0) continue;
    const int KP = (K + T::KS - 1) / T::KS * T::KS;
    if (transA) {
      for (int e = tid; e < K * rows; e += 256) {
        const int kk = e / rows, r = e - kk * rows;
        As[r * ALD + kk] = mf_a(Ap[e]);
      }
      for (int e = tid; e < rows * (KP - K); e += 256) {
        const int r = e / (KP - K), kk = K + e - r * (KP - K);
        As[r * ALD + kk] = SA(0);
      }
    } else {
      for (int e = tid; e < rows * KP; e += 256) {
        const int r = e / KP, kk = e - r * KP;
        As[r * ALD + kk] = kk < K ? mf_a(Ap[(size_t)r * K + kk]) : SA(0);
      }
    }
    for (int e = tid; e < KP * NC; e += 256) {
      const int v = e / KP, kk = e - v * KP;
      const SB val = (kk < K && v < nvc) ? mf_b<SB, V>(Bp[(size_t)v * ldb + kk]) : SB(0);
      if (BF) Bs[v * BLD + kk] = val;
      else Bs[kk * BLD + v] = val;
    }
    __syncthreads();
    if (16 * wave < rows) {
      const int ar = (16 * wave + (lane & 15)) * ALD;
      for (int k0 = 0; k0 < KP; k0 += T::KS) {
        if constexpr (BF) {
          const mf_s4 a = *reinterpret_cast<const mf_s4*>(&As[ar + k0 + 4 * (lane >> 4)]);
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) {
            const mf_s4 b = *reinterpret_cast<const mf_s4*>(
                &Bs[(ct * 16 + (lane & 15)) * BLD + k0 + 4 * (lane >> 4)]);
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[ct], 0, 0, 0);
          }
        } else {
          const SA a = As[ar + k0 + (lane >> 4)];
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) {
            const SB b = Bs[(k0 + (lane >> 4)) * BLD + ct * 16 + (lane & 15)];
            if constexpr (sizeof(SA) == 8)
              acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[ct], 0, 0, 0);
            else
              acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[ct], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
}

// row of output tile element held in register r: column lane % 16, row
// 4 (lane / 16) + r for the f32 products, 4 r + lane / 16 for the f64 product
template <class M>
__device__ inline int mf_row(int r, int lane) {
  return sizeof(typename MfmaTraits<M>::SA) == 8 ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r;
}

#define MF_SHARED(M, NT)                                                                    \
  using T_ = MfmaTraits<M>;                                                                 \
  constexpr int NC_ = 16 * (NT);                                                            \
  constexpr int BLD_ = T_::KS == 16 ? 64 + T_::PADB : NC_ + T_::PADB;                       \
  __shared__ __align__(16) typename T_::SA As[LEAF_MAX * T_::ALD];                          \
  __shared__ __align__(16) typename T_::SB Bs[T_::KS == 16 ? NC_ * BLD_ : LEAF_MAX * BLD_]; \
  typename T_::Acc acc[NT];

// leaf stage: y_t = alpha (U_t y^_t + sum_near D_ts x_s) + beta y_t
template <class M, class V, int NT>
__global__ __launch_bounds__(256) void k_leaf_mfma(
    int L, const int32_t* __restrict__ cstart, const int32_t* __restrict__ csize,
    const int32_t* __restrict__ rank, const int64_t* __restrict__ kpre,
    const int64_t* __restrict__ Uoff, const M* __restrict__ U,
    const int32_t* __restrict__ near_ptr, const int32_t* __restrict__ near_col,
    const int64_t* __restrict__ Doff, const M* __restrict__ D, int nv, const V* __restrict__ yh,
    const V* __restrict__ x, int ldx, V alpha, V beta, V* __restrict__ y, int ldy) {
  MF_SHARED(M, NT)
  const int i = xcd_local(blockIdx.x, gridDim.x);
  const int leaf_base = (1 << L) - 1;
  const int c = leaf_base + i;
  const int r0 = cstart[c], m = csize[c];
  const int v0 = blockIdx.y * NC_;
  const int nvc = min(NC_, nv - v0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = rank[c];
  const int g0 = near_ptr[i], nnear = near_ptr[i + 1] - g0;
  auto src = [&](int q, const M*& Ap, int& K, bool& tA, const V*& Bp, int& ldb) {
    tA = false;
    if (q < nnear) {
      const int g = g0 + q;
      const int sc = leaf_base + near_col[g];
      Ap = D + Doff[g];
      K = csize[sc];
      Bp = x + (size_t)v0 * ldx + cstart[sc];
      ldb = ldx;
    } else {
      Ap = U + Uoff[i];
      K = k;
      Bp = yh + kpre[c] * nv + (size_t)v0 * k;
      ldb = k;
    }
  };
  blockrow_mfma<M, V, NT>(m, nnear + (k > 0 ? 1 : 0), src, nvc, acc, As, Bs);
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * wave + mf_row<M>(r, lane), col = ct * 16 + (lane & 15);
      if (row < m && col < nvc) {
        V* yp = y + (size_t)(v0 + col) * ldy + r0 + row;
        const V val = alpha * (V)acc[ct][r];
        *yp = beta == V(0) ? val : val + beta * *yp;
      }
    }
}

// Block-row product in FP64 or FP32, pipelined through LDS: out (rows x nvc)
// = sum over sources q of A_q B_q (A_q row-major rows x K_q, B_q
// column-major K_q x nvc with leading dimension ldb_q; rows, K_q <= 64).
// Each source is read with coalesced loads (A a row at a time, B a column at
// a time) into registers two sources ahead of its use, stored into one of two
// LDS tile buffers, and multiplied on the matrix cores (16x16x4, f64 or f32)
// from there after a single barrier, so that the loads of the next sources
// overlap the products of this one.  The products and their order are those
// of blockrow_mfma (sources ascending, k ascending in steps of 4); wave w owns
// rows 16 w..16 w + 15 and NT 16-column tiles.
// (global-memory pointers: their loads then count only against the vector
// memory counter, not against the LDS one that the tile accesses wait on)
template <class T> using gptr_t = const T __attribute__((address_space(1)))*;
template <class T> struct PipeSrc {
  gptr_t<T> A;
  gptr_t<T> B;
  int K, ldb;
};
template <class T> struct PipeMfma;
template <> struct PipeMfma<double> {
  using Acc = mf_d4;
  static constexpr int PAD = 2;   // row padding of the tiles (bank spread)
  __device__ static Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct PipeMfma<float> {
  using Acc = mf_f4;
  static constexpr int PAD = 4;
  __device__ static Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
constexpr int PIPE_MAXSRC = 64;
template <class T, int NT> struct PipeTiles {
  static constexpr int NC = 16 * NT, ALD = 64 + PipeMfma<T>::PAD, BLD = NC + PipeMfma<T>::PAD;
  static constexpr int RA = 16, RB = NC / 4;    // registers per thread
  T A[2][64 * ALD];
  T B[2][64 * BLD];
};

template <class T, int NT>
__device__ inline void blockrow_lds_pipe(int rows, int nsrc, const PipeSrc<T>* __restrict__ ps,
                                         int nvc, typename PipeMfma<T>::Acc (&acc)[NT],
                                         PipeTiles<T, NT>& tl) {
  using P = PipeTiles<T, NT>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // A: wave w, register j holds row 4 j + w, k = lane (one row of the
  // row-major block per load instruction); B: register j holds column
  // 4 j + w, k = lane (one column per instruction).  Loads use clamped,
  // in-range addresses; the positions outside the block are zeroed when
  // stored to LDS.
  auto gload = [&](int q, T (&ra)[P::RA], T (&rb)[P::RB]) {
    // (straight-line loads: an empty block, K = 0, carries pointers to valid
    // memory and reads its first element, stored as zeros)
    const PipeSrc<T> S = ps[q < nsrc ? q : nsrc - 1];
    const int kl = (S.K > 0 ? S.K : 1) - 1;
    const int kc = lane < kl ? lane : kl;
#pragma unroll
    for (int j = 0; j < P::RA; ++j) {
      const int r = 4 * j + wave;
      ra[j] = S.A[(size_t)(r < rows ? r : rows - 1) * S.K + kc];
    }
#pragma unroll
    for (int j = 0; j < P::RB; ++j) {
      const int cb = 4 * j + wave;
      rb[j] = S.B[(size_t)(cb < nvc ? cb : nvc - 1) * S.ldb + kc];
    }
  };
  auto lstore = [&](int q, int buf, const T (&ra)[P::RA], const T (&rb)[P::RB]) {
    const int K = q < nsrc ? ps[q].K : 0;
#pragma unroll
    for (int j = 0; j < P::RA; ++j) {
      const int r = 4 * j + wave;
      tl.A[buf][r * P::ALD + lane] = (r < rows && lane < K) ? ra[j] : T(0);
    }
#pragma unroll
    for (int j = 0; j < P::RB; ++j) {
      const int cb = 4 * j + wave;
      tl.B[buf][lane * P::BLD + cb] = (cb < nvc && lane < K) ? rb[j] : T(0);
    }
  };
  // the k-steps in groups of four (16 k-values), each group's LDS reads
  // issued together ahead of its products; groups wholly past K are skipped
  auto mma = [&](int q, int buf) {
    if (16 * wave >= rows || q >= nsrc) return;
    const int KP = (ps[q].K + 3) & ~3;
    const T* As = tl.A[buf] + (16 * wave + (lane & 15)) * P::ALD + (lane >> 4);
    const T* Bs = tl.B[buf] + (lane >> 4) * P::BLD + (lane & 15);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (16 * g >= KP) break;
      T a[4], b[NT][4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = As[16 * g + 4 * t];
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) b[ct][t] = Bs[(16 * g + 4 * t) * P::BLD + 16 * ct];
      }
      // (a group always takes its four k-steps: the tiles are zero past K,
      // so the extra steps add exact zeros)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) acc[ct] = PipeMfma<T>::mma(a[t], b[ct][t], acc[ct]);
    }
  };
  if (nsrc <= 0) return;
  T ra0[P::RA], rb0[P::RB], ra1[P::RA], rb1[P::RB];
  gload(0, ra0, rb0);
  gload(1, ra1, rb1);
  // (sources in pairs, an odd count padded by an empty one: the loop body
  // has no exit in the middle, so each register set keeps its place)
  for (int q = 0; q < nsrc; q += 2) {
    // buffer 0 was last read by the products of source q - 2, which every
    // wave finished before the barrier of source q - 1
    lstore(q, 0, ra0, rb0);
    __syncthreads();
    gload(q + 2, ra0, rb0);
    mma(q, 0);
    lstore(q + 1, 1, ra1, rb1);
    __syncthreads();
    gload(q + 3, ra1, rb1);
    mma(q + 1, 1);
  }
}

// The same pipeline for BF16 storage with FP32 vectors: 16x16x16 BF16
// products with FP32 accumulation (four consecutive k per lane and product),
// A tiles row-major and B tiles column-major per vector (a lane's four k
// contiguous), the vectors rounded to BF16 when stored to LDS; the products
// and their order are those of blockrow_mfma's BF16 path.
struct PipeSrcBF {
  gptr_t<uint16_t> A;   // BF16 bits
  gptr_t<float> B;
  int K, ldb;
};
template <int NT> struct PipeTilesBF {
  static constexpr int NC = 16 * NT, LD = 64 + 8;
  static constexpr int RA = 16, RB = NC / 4;
  uint16_t A[2][64 * LD];
  uint16_t B[2][NC * LD];
};

template <int NT>
__device__ inline void blockrow_lds_pipe_bf(int rows, int nsrc, const PipeSrcBF* __restrict__ ps,
                                            int nvc, mf_f4 (&acc)[NT], PipeTilesBF<NT>& tl) {
  using P = PipeTilesBF<NT>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto gload = [&](int q, uint16_t (&ra)[P::RA], float (&rb)[P::RB]) {
    const PipeSrcBF S = ps[q < nsrc ? q : nsrc - 1];
    const int kl = (S.K > 0 ? S.K : 1) - 1;
    const int kc = lane < kl ? lane : kl;
#pragma unroll
    for (int j = 0; j < P::RA; ++j) {
      const int r = 4 * j + wave;
      ra[j] = S.A[(size_t)(r < rows ? r : rows - 1) * S.K + kc];
    }
#pragma unroll
    for (int j = 0; j < P::RB; ++j) {
      const int cb = 4 * j + wave;
      rb[j] = S.B[(size_t)(cb < nvc ? cb : nvc - 1) * S.ldb + kc];
    }
  };
  auto lstore = [&](int q, int buf, const uint16_t (&ra)[P::RA], const float (&rb)[P::RB]) {
    const int K = q < nsrc ? ps[q].K : 0;
#pragma unroll
    for (int j = 0; j < P::RA; ++j) {
      const int r = 4 * j + wave;
      tl.A[buf][r * P::LD + lane] = (r < rows && lane < K) ? ra[j] : (uint16_t)0;
    }
#pragma unroll
    for (int j = 0; j < P::RB; ++j) {
      const int cb = 4 * j + wave;
      tl.B[buf][cb * P::LD + lane] = (cb < nvc && lane < K) ? float_to_bf16(rb[j]).bits : (uint16_t)0;
    }
  };
  auto mma = [&](int q, int buf) {
    if (16 * wave >= rows || q >= nsrc) return;
    const int KP = (ps[q].K + 15) & ~15;
    const uint16_t* As = tl.A[buf] + (16 * wave + (lane & 15)) * P::LD + 4 * (lane >> 4);
    const uint16_t* Bs = tl.B[buf] + (lane & 15) * P::LD + 4 * (lane >> 4);
    mf_s4 a[4], b[NT][4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      a[g] = *reinterpret_cast<const mf_s4*>(As + 16 * g);
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) b[ct][g] = *reinterpret_cast<const mf_s4*>(Bs + 16 * ct * P::LD + 16 * g);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (16 * g >= KP) break;
#pragma unroll
      for (int ct = 0; ct < NT; ++ct)
        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[g], b[ct][g], acc[ct], 0, 0, 0);
    }
  };
  if (nsrc <= 0) return;
  uint16_t ra0[P::RA], ra1[P::RA];
  float rb0[P::RB], rb1[P::RB];
  gload(0, ra0, rb0);
  gload(1, ra1, rb1);
  for (int q = 0; q < nsrc; q += 2) {
    lstore(q, 0, ra0, rb0);
    __syncthreads();
    gload(q + 2, ra0, rb0);
    mma(q, 0);
    lstore(q + 1, 1, ra1, rb1);
    __syncthreads();
    gload(q + 3, ra1, rb1);
    mma(q + 1, 1);
  }
}

// leaf stage in FP64 or FP32: y_t = alpha (U_t y^_t + sum_near D_ts x_s) + beta y_t
// Split far lists: when the coupling stage has few output tiles, each tile's
// list of blocks is cut into G consecutive groups taken by G workgroups
// (blockIdx.z), which store partial sums; the last to arrive adds the G
// partials in group order, so the sums do not depend on arrival order or on
// the tile width.  Publication as in the block Jacobi: every wave's stores
// complete at the L2, thread 0 fences at device scope before it increments
// the tile's counter, and the last workgroup resets the counter and fences
// again before its waves read the other partials.
template <class V>
struct Split {
  int G = 1;            // groups per block row
  V* part = nullptr;    // the G partial outputs, pstride elements apart
  int64_t pstride = 0;
  int* cnt = nullptr;   // arrival counters, one per output tile, zero between products
};

__device__ inline bool split_last(int* cnt, int G) {
  __shared__ int last;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const int old = atomicAdd(cnt, 1);
    last = old == G - 1;
    if (last) {
      atomicExch(cnt, 0);
      __threadfence();
    }
  }
  __syncthreads();
  return last != 0;
}

template <class M, class V, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_leaf_direct(
    int L, const int32_t* __restrict__ cstart, const int32_t* __restrict__ csize,
    const int32_t* __restrict__ rank, const int64_t* __restrict__ kpre,
    const int64_t* __restrict__ Uoff, const M* __restrict__ U,
    const int32_t* __restrict__ near_ptr, const int32_t* __restrict__ near_col,
    const int64_t* __restrict__ Doff, const M* __restrict__ D, int nv, const V* __restrict__ yh,
    const V* __restrict__ x, int ldx, V alpha, V beta, V* __restrict__ y, int ldy) {
  constexpr bool BF = std::is_same<M, bf16_t>::value;
  static_assert((std::is_same<M, V>::value &&
                 (std::is_same<M, double>::value || std::is_same<M, float>::value)) ||
                    (BF && std::is_same<V, float>::value),
                "FP64 or FP32 storage and vectors, or BF16 storage with FP32 vectors");
  using T = typename std::conditional<BF, float, M>::type;   // vector / accumulator type
  using AT = typename std::conditional<BF, uint16_t, M>::type;
  using Src = typename std::conditional<BF, PipeSrcBF, PipeSrc<T>>::type;
  using Tiles = typename std::conditional<BF, PipeTilesBF<NT>, PipeTiles<T, NT>>::type;
  constexpr int NC = 16 * NT;
  __shared__ Src ps[PIPE_MAXSRC];
  __shared__ Tiles tl;
  const int i = xcd_local(blockIdx.x, gridDim.x);
  const int leaf_base = (1 << L) - 1;
  const int c = leaf_base + i;
  const int r0 = cstart[c], m = csize[c];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int v0 = blockIdx.y * NC;
  const int nvc = min(NC, nv - v0);
  const int k = rank[c];
  const int g0 = near_ptr[i], nnear = near_ptr[i + 1] - g0;
  const int nsrc = nnear + (k > 0 ? 1 : 0);
  typename PipeMfma<T>::Acc acc[NT];
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[ct][r] = 0;
  for (int q0 = 0; q0 < nsrc; q0 += PIPE_MAXSRC) {
    const int nb = min(PIPE_MAXSRC, nsrc - q0);
    __syncthreads();
    if ((int)threadIdx.x < nb) {
      const int q = q0 + (int)threadIdx.x;
      Src d;
      if (q < nnear) {
        const int g = g0 + q;
        const int sc = leaf_base + near_col[g];
        d.A = (gptr_t<AT>)(const AT*)(D + Doff[g]);
        d.K = csize[sc];
        d.B = (gptr_t<T>)(x + (size_t)v0 * ldx + cstart[sc]);
        d.ldb = ldx;
      } else {
        d.A = (gptr_t<AT>)(const AT*)(U + Uoff[i]);
        d.K = k;
        d.B = (gptr_t<T>)(yh + kpre[c] * nv + (size_t)v0 * k);
        d.ldb = k;
      }
      ps[threadIdx.x] = d;
    }
    __syncthreads();
    if constexpr (BF) blockrow_lds_pipe_bf<NT>(m, nb, ps, nvc, acc, tl);
    else blockrow_lds_pipe<T, NT>(m, nb, ps, nvc, acc, tl);
  }
  if (16 * wave >= m) return;
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * wave + mf_row<M>(r, lane), col = ct * 16 + (lane & 15);
      if (row < m && col < nvc) {
        V* yp = y + (size_t)(v0 + col) * ldy + r0 + row;
        const V val = alpha * (V)acc[ct][r];
        *yp = beta == V(0) ? val : val + beta * *yp;
      }
    }
}

// upsweep at the leaves: x^_t = U_t^T x_t (k_t x nv)
template <class M, class V, int NT>
__global__ __launch_bounds__(256) void k_up_leaf_mfma(
    int L, const int32_t* __restrict__ cstart, const int32_t* __restrict__ csize,
    const int32_t* __restrict__ rank, const int64_t* __restrict__ kpre,
    const int64_t* __restrict__ Uoff, const M* __restrict__ U, const V* __restrict__ x, int ldx,
    int nv, V* __restrict__ xh) {
  MF_SHARED(M, NT)
  const int i = blockIdx.x;
  const int c = (1 << L) - 1 + i;
  const int k = rank[c];
  if (k == 0) return;
  const int v0 = blockIdx.y * NC_;
  const int nvc = min(NC_, nv - v0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto src = [&](int, const M*& Ap, int& K, bool& tA, const V*& Bp, int& ldb) {
    Ap = U + Uoff[i];
    K = csize[c];
    tA = true;
    Bp = x + (size_t)v0 * ldx + cstart[c];
    ldb = ldx;
  };
  blockrow_mfma<M, V, NT>(k, 1, src, nvc, acc, As, Bs);
  V* out = xh + kpre[c] * nv;
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * wave + mf_row<M>(r, lane), col = ct * 16 + (lane & 15);
      if (row < k && col < nvc) out[(size_t)(v0 + col) * k + row] = (V)acc[ct][r];
    }
}

// couplings: y^_t = sum_{s in far(t)} S_ts x^_s for every non-root cluster
template <class M, class V, int NT>
__global__ __launch_bounds__(256) void k_coupling_mfma(
    const int32_t* __restrict__ rank, const int64_t* __restrict__ kpre,
    const int32_t* __restrict__ far_ptr, const int32_t* __restrict__ far_col,
    const int64_t* __restrict__ Soff, const M* __restrict__ S, int nv, const V* __restrict__ xh,
    V* __restrict__ yh, Split<V> sp) {
  MF_SHARED(M, NT)
  const int c = blockIdx.x + 1;
  const int kt = rank[c];
  if (kt == 0) return;
  const int l = 31 - __clz(c + 1);
  const int base = (1 << l) - 1;
  // this workgroup's group of the far partners (all of them when G = 1)
  const int G = sp.G;
  const int f0 = far_ptr[c + l], nf = far_ptr[c + l + 1] - f0, chunk = (nf + G - 1) / G;
  const int pb = f0 + min(nf, (int)blockIdx.z * chunk), pe = f0 + min(nf, ((int)blockIdx.z + 1) * chunk);
  const int v0 = blockIdx.y * NC_;
  const int nvc = min(NC_, nv - v0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto src = [&](int q, const M*& Ap, int& K, bool& tA, const V*& Bp, int& ldb) {
    const int g = pb + q;
    const int cs = base + far_col[g];
    tA = false;
    K = rank[cs];
    Ap = S + Soff[g];
    Bp = xh + kpre[cs] * nv + (size_t)v0 * K;
    ldb = K;
  };
  blockrow_mfma<M, V, NT>(kt, pe - pb, src, nvc, acc, As, Bs);
  V* out = yh + kpre[c] * nv;
  V* dst = G == 1 ? out : sp.part + blockIdx.z * sp.pstride + kpre[c] * nv;
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * wave + mf_row<M>(r, lane), col = ct * 16 + (lane & 15);
      if (row < kt && col < nvc) dst[(size_t)(v0 + col) * kt + row] = (V)acc[ct][r];
    }
  if (G == 1 || !split_last(sp.cnt + (size_t)blockIdx.x * gridDim.y + blockIdx.y, G)) return;
  const V* p0 = sp.part + kpre[c] * nv;
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * wave + mf_row<M>(r, lane), col = ct * 16 + (lane & 15);
      if (row < kt && col < nvc) {
        const size_t e = (size_t)(v0 + col) * kt + row;
        V sum = p0[e];
        for (int z = 1; z < G; ++z) sum += p0[z * sp.pstride + e];
        out[e] = sum;
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

// nested-basis transfers on matrix cores, one workgroup per (cluster, NC
// vectors).  Upsweep: x^_p = E_c1^T x^_c1 + E_c2^T x^_c2 for the parents p of
// level l (E_c row-major k_c x k_p, taken transposed).  Downsweep:
// y^_c += E_c y^_p for the clusters c of level l.  Ranks <= 64.
template <class M, class V, int NT>
__global__ __launch_bounds__(256) void k_up_transfer_mfma(int l, const int32_t* __restrict__ rank,
                                                          const int64_t* __restrict__ kpre,
                                                          const int64_t* __restrict__ Eoff,
                                                          const M* __restrict__ E, int nv,
                                                          V* __restrict__ xh) {
  MF_SHARED(M, NT)
  const int p = blockIdx.x;
  const int cp = (1 << l) - 1 + p;
  const int kp = rank[cp];
  if (kp == 0) return;
  const int c1 = (1 << (l + 1)) - 1 + 2 * p;
  const int v0 = blockIdx.y * NC_;
  const int nvc = min(NC_, nv - v0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto src = [&](int q, const M*& Ap, int& K, bool& tA, const V*& Bp, int& ldb) {
    const int c = c1 + q;
    tA = true;
    K = rank[c];
    Ap = E + Eoff[c];
    Bp = xh + kpre[c] * nv + (size_t)v0 * K;
    ldb = K;
  };
  blockrow_mfma<M, V, NT>(kp, 2, src, nvc, acc, As, Bs);
  V* out = xh + kpre[cp] * nv;
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * wave + mf_row<M>(r, lane), col = ct * 16 + (lane & 15);
      if (row < kp && col < nvc) out[(size_t)(v0 + col) * kp + row] = (V)acc[ct][r];
    }
}

template <class M, class V, int NT>
__global__ __launch_bounds__(256) void k_down_transfer_mfma(int l, const int32_t* __restrict__ rank,
                                                            const int64_t* __restrict__ kpre,
                                                            const int64_t* __restrict__ Eoff,
                                                            const M* __restrict__ E, int nv,
                                                            V* __restrict__ yh) {
  MF_SHARED(M, NT)
  const int ch = blockIdx.x;
  const int cc = (1 << l) - 1 + ch;
  const int cp = (1 << (l - 1)) - 1 + ch / 2;
  const int kc = rank[cc], kp = rank[cp];
  if (kc == 0 || kp == 0) return;
  const int v0 = blockIdx.y * NC_;
  const int nvc = min(NC_, nv - v0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto src = [&](int q, const M*& Ap, int& K, bool& tA, const V*& Bp, int& ldb) {
    (void)q;
    tA = false;
    K = kp;
    Ap = E + Eoff[cc];
    Bp = yh + kpre[cp] * nv + (size_t)v0 * kp;
    ldb = kp;
  };
  blockrow_mfma<M, V, NT>(kc, 1, src, nvc, acc, As, Bs);
  V* out = yh + kpre[cc] * nv;
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * wave + mf_row<M>(r, lane), col = ct * 16 + (lane & 15);
      if (row < kc && col < nvc) out[(size_t)(v0 + col) * kc + row] += (V)acc[ct][r];
    }
}

// ------------------------------------------------------------------ drivers
template <class M, class V>
static constexpr bool has_mfma() {
  return (std::is_same<M, double>::value && std::is_same<V, double>::value) ||
         (std::is_same<M, float>::value && std::is_same<V, float>::value) ||
         (std::is_same<M, bf16_t>::value && std::is_same<V, float>::value);
}

// launches of the matrix-core stages with NT 16-column tiles per workgroup
template <class M, class V, int NT>
static void up_leaf_nt(const h2_matrix* A, int nv, const V* xt, int ldx, V* xh, hipStream_t s) {
  const h2_tree* t = A->tree;
  const unsigned gy = (unsigned)((nv + 16 * NT - 1) / (16 * NT));
  k_up_leaf_mfma<M, V, NT><<<dim3(1 << t->L, gy), 256, 0, s>>>(
      t->L, t->d_cstart.as<int32_t>(), t->d_csize.as<int32_t>(), A->d_rank.as<int32_t>(),
      A->d_kpre.as<int64_t>(), A->d_U_off.as<int64_t>(), A->st.U.as<M>(), xt, ldx, nv, xh);
}
template <class M, class V, int NT>
static void coupling_nt(const h2_matrix* A, int nv, const V* xh, V* yh, hipStream_t s,
                        Split<V> sp) {
  const h2_tree* t = A->tree;
  const unsigned gy = (unsigned)((nv + 16 * NT - 1) / (16 * NT));
  // (small blocks, many per cluster: the single-buffered LDS tiles of
  // blockrow_mfma, which leave room for two workgroups per compute unit, beat
  // the register-pipelined product here, in FP64 too)
  k_coupling_mfma<M, V, NT><<<dim3(t->nclusters() - 1, gy, sp.G), 256, 0, s>>>(
      A->d_rank.as<int32_t>(), A->d_kpre.as<int64_t>(), t->d_far_ptr.as<int32_t>(),
      t->d_far_col.as<int32_t>(), A->d_S_off.as<int64_t>(), A->st.S.as<M>(), nv, xh, yh, sp);
}
template <class M, class V, int NT>
static void leaf_nt(const h2_matrix* A, int nv, V alpha, const V* xt, int ldx, V beta, V* yt,
                    int ldy, const V* yh, hipStream_t s) {
  const h2_tree* t = A->tree;
  const unsigned gy = (unsigned)((nv + 16 * NT - 1) / (16 * NT));
  // the LDS-pipelined kernel (FP64, FP32, and BF16 storage with FP32 vectors)
  if constexpr ((std::is_same<M, V>::value &&
                 (std::is_same<M, double>::value || std::is_same<M, float>::value)) ||
                (std::is_same<M, bf16_t>::value && std::is_same<V, float>::value))
    k_leaf_direct<M, V, NT><<<dim3(1 << t->L, gy), 256, 0, s>>>(
        t->L, t->d_cstart.as<int32_t>(), t->d_csize.as<int32_t>(), A->d_rank.as<int32_t>(),
        A->d_kpre.as<int64_t>(), A->d_U_off.as<int64_t>(), A->st.U.as<M>(),
        t->d_near_ptr.as<int32_t>(), t->d_near_col.as<int32_t>(), A->d_D_off.as<int64_t>(),
        A->st.D.as<M>(), nv, yh, xt, ldx, alpha, beta, yt, ldy);
  else
    k_leaf_mfma<M, V, NT><<<dim3(1 << t->L, gy), 256, 0, s>>>(
        t->L, t->d_cstart.as<int32_t>(), t->d_csize.as<int32_t>(), A->d_rank.as<int32_t>(),
        A->d_kpre.as<int64_t>(), A->d_U_off.as<int64_t>(), A->st.U.as<M>(),
        t->d_near_ptr.as<int32_t>(), t->d_near_col.as<int32_t>(), A->d_D_off.as<int64_t>(),
        A->st.D.as<M>(), nv, yh, xt, ldx, alpha, beta, yt, ldy);
}

__global__ void k_zero_i32(int* p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0;
}

// groups per far list of the coupling stage: split only where the couplings
// are large (mean rank of at least 32: a list's chain of k x k products is
// long next to the cost of the partial sums) and the tiles at the narrowest
// width (16 vectors) are too few to fill the chip (about 2048 workgroups).
// Independent of the chosen width, so every width sums alike.
static int split_groups(int64_t tiles, double mean_rank) {
  if (mean_rank < 32.0 || tiles >= 2048) return 1;
  return (int)std::min<int64_t>(4, (2048 + tiles - 1) / tiles);
}

// coef: 2 * (sum of ranks) * nv coefficient words (x-hat, y-hat); nullptr:
// the matrix's own workspace, grown on demand, which also holds the partial
// sums of split far lists (coef given: no split)
template <class M, class V>
static void gemv_tree_run(const h2_matrix* A, int nv, V alpha, const V* xt, int ldx, V beta,
                          V* yt, int ldy, hipStream_t s, int nt, V* coef = nullptr) {
  const h2_tree* t = A->tree;
  const int L = t->L;
  const int64_t ktot = A->kpre.back();
  const int64_t gy1 = (nv + 15) / 16;
  Split<V> spc;   // coupling stage
  if (!coef) {
    if (nt > 0 && L >= 1)
      spc.G = split_groups((int64_t)(t->nclusters() - 1) * gy1, (double)ktot / (t->nclusters() - 1));
    const int64_t wc = spc.G > 1 ? spc.G * ktot * nv : 0;
    const size_t need = (size_t)(2 * ktot * nv + wc) * sizeof(V);
    A->ws.reserve(std::max<size_t>(need, 256));
    coef = A->ws.as<V>();
    spc.part = coef + 2 * ktot * nv;
    spc.pstride = ktot * nv;
    if (spc.G > 1) {
      // arrival counters, one per coupling tile (zero at rest)
      const int64_t nc = (int64_t)t->nclusters() * gy1;
      if ((size_t)nc * sizeof(int) > A->ws_cnt.bytes) {
        A->ws_cnt.alloc((size_t)nc * sizeof(int));
        k_zero_i32<<<(unsigned)((nc + 255) / 256), 256, 0, s>>>(A->ws_cnt.as<int>(), nc);
      }
      spc.cnt = A->ws_cnt.as<int>();
    }
  }
  V* xh = coef;
  V* yh = xh + ktot * nv;
  const M* U = A->st.U.as<M>();
  const M* E = A->st.E.as<M>();
  const M* S = A->st.S.as<M>();
  const M* D = A->st.D.as<M>();
  const int32_t* rank = A->d_rank.as<int32_t>();
  const int64_t* kpre = A->d_kpre.as<int64_t>();
  const int32_t* cstart = t->d_cstart.as<int32_t>();
  const int32_t* csize = t->d_csize.as<int32_t>();
  // matrix cores for the dense contractions when every block fits the 64 x 64 tiles
  // (leaves are at most 64 points; ranks above 64 take the scalar kernels)
  const bool mf = nt > 0;
  if (ktot > 0 && L >= 1) {
    if constexpr (has_mfma<M, V>()) {
      if (nt == 1) up_leaf_nt<M, V, 1>(A, nv, xt, ldx, xh, s);
      else if (nt == 2) up_leaf_nt<M, V, 2>(A, nv, xt, ldx, xh, s);
      else if (nt == 4) up_leaf_nt<M, V, 4>(A, nv, xt, ldx, xh, s);
    }
    if (!mf)
      k_up_leaf<M, V><<<1 << L, 256, 0, s>>>(L, cstart, csize, rank, kpre,
                                              A->d_U_off.as<int64_t>(), U, xt, ldx, nv, xh);
    for (int l = L - 1; l >= 1; --l) {
      if constexpr (has_mfma<M, V>()) {
        if (mf) {
          const unsigned gy = (unsigned)((nv + 16 * nt - 1) / (16 * nt));
          if (nt == 1) k_up_transfer_mfma<M, V, 1><<<dim3(1 << l, gy), 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv, xh);
          else if (nt == 2) k_up_transfer_mfma<M, V, 2><<<dim3(1 << l, gy), 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv, xh);
          else k_up_transfer_mfma<M, V, 4><<<dim3(1 << l, gy), 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv, xh);
          continue;
        }
      }
      k_up_transfer<M, V><<<1 << l, 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv,
                                                  xh);
    }
    if constexpr (has_mfma<M, V>()) {
      if (nt == 1) coupling_nt<M, V, 1>(A, nv, xh, yh, s, spc);
      else if (nt == 2) coupling_nt<M, V, 2>(A, nv, xh, yh, s, spc);
      else if (nt == 4) coupling_nt<M, V, 4>(A, nv, xh, yh, s, spc);
    }
    if (!mf)
      k_coupling<M, V><<<t->nclusters() - 1, 256, 0, s>>>(
          rank, kpre, t->d_far_ptr.as<int32_t>(), t->d_far_col.as<int32_t>(),
          A->d_S_off.as<int64_t>(), S, nv, xh, yh);
    for (int l = 2; l <= L; ++l) {
      if constexpr (has_mfma<M, V>()) {
        if (mf) {
          const unsigned gy = (unsigned)((nv + 16 * nt - 1) / (16 * nt));
          if (nt == 1) k_down_transfer_mfma<M, V, 1><<<dim3(1 << l, gy), 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv, yh);
          else if (nt == 2) k_down_transfer_mfma<M, V, 2><<<dim3(1 << l, gy), 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv, yh);
          else k_down_transfer_mfma<M, V, 4><<<dim3(1 << l, gy), 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv, yh);
          continue;
        }
      }
      k_down_transfer<M, V><<<1 << l, 256, 0, s>>>(l, rank, kpre, A->d_E_off.as<int64_t>(), E, nv,
                                                    yh);
    }
  }
  if constexpr (has_mfma<M, V>()) {
    if (nt == 1) leaf_nt<M, V, 1>(A, nv, alpha, xt, ldx, beta, yt, ldy, yh, s);
    else if (nt == 2) leaf_nt<M, V, 2>(A, nv, alpha, xt, ldx, beta, yt, ldy, yh, s);
    else if (nt == 4) leaf_nt<M, V, 4>(A, nv, alpha, xt, ldx, beta, yt, ldy, yh, s);
  }
  if (!mf) {
    dim3 grid(1 << L, (nv + NVC - 1) / NVC);
    k_leaf_out<M, V><<<grid, 256, 0, s>>>(L, cstart, csize, rank, kpre, A->d_U_off.as<int64_t>(), U,
                                          t->d_near_ptr.as<int32_t>(), t->d_near_col.as<int32_t>(),
                                          A->d_D_off.as<int64_t>(), D, nv, yh, xt, ldx, alpha,
                                          beta, yt, ldy);
  }
  H2_LAUNCH_CHECK();
}

// Tile-width autotuner: on the first product on a tree with a given class of
// vector counts (ceil(nv / 16), capped at 4) and precisions, every width of
// 16, 32 or 64 vectors per workgroup that the count can use is timed with HIP
// events (two runs each into a scratch output, after one untimed run) and the
// fastest is kept with the tree for the matrices built on it.
// Under stream capture nothing is timed and a width from the vector count
// is used instead.  Every width gives the same result (the same products
// summed in the same order).
template <class M, class V>
static int tile_width(const h2_matrix* A, int nv, const V* xt, int ldx, hipStream_t s) {
  if (!(has_mfma<M, V>() && A->kmax <= LEAF_MAX)) return 0;
  const std::tuple<int, int, int> key{std::min((nv + 15) / 16, 4), (int)sizeof(M), (int)sizeof(V)};
  auto it = A->tree->tuned_nt.find(key);
  if (it != A->tree->tuned_nt.end()) return it->second;
  const int heur = nv <= 16 ? 1 : (nv <= 32 ? 2 : 4);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  H2_HIP(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return heur;
  const int n = A->tree->n;
  DevBuf ytmp((size_t)n * nv * sizeof(V));
  hipEvent_t e0, e1;
  H2_HIP(hipEventCreate(&e0));
  H2_HIP(hipEventCreate(&e1));
  int best = heur;
  float best_ms = 1e30f;
  for (int nt : {1, 2, 4}) {
    if (nt > 1 && 16 * (nt / 2) >= nv) break;   // wider tiles would only add padding
    gemv_tree_run<M, V>(A, nv, V(1), xt, ldx, V(0), ytmp.as<V>(), n, s, nt);
    H2_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 2; ++r) gemv_tree_run<M, V>(A, nv, V(1), xt, ldx, V(0), ytmp.as<V>(), n, s, nt);
    H2_HIP(hipEventRecord(e1, s));
    H2_HIP(hipEventSynchronize(e1));
    float ms = 0;
    H2_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) { best_ms = ms; best = nt; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  A->tree->tuned_nt[key] = best;
  if (verbose()) std::fprintf(stderr, "  [hgemv] n %d nv %d: tile width %d vectors\n", n, nv, 16 * best);
  return best;
}

template <class M, class V>
static void gemv_tree_impl(const h2_matrix* A, int nv, V alpha, const V* xt, int ldx, V beta,
                           V* yt, int ldy, hipStream_t s, int nt_force) {
  int nt = 0;
  if (has_mfma<M, V>() && A->kmax <= LEAF_MAX) {
    H2_CHECK(nt_force == 0 || nt_force == 1 || nt_force == 2 || nt_force == 4, H2_EINVAL,
             "tile width must be 1, 2 or 4 tiles");
    nt = nt_force ? nt_force : tile_width<M, V>(A, nv, xt, ldx, s);
  }
  gemv_tree_run<M, V>(A, nv, alpha, xt, ldx, beta, yt, ldy, s, nt);
}

void gemv_tree_f64(const h2_matrix* A, int nv, double alpha, const double* xt, int ldx,
                   double beta, double* yt, int ldy, hipStream_t s, int nt_force) {
  if (nv <= 0) return;
  H2_CHECK(A->st.prec == H2_FP64, H2_EINVAL, "FP64 HGEMV needs an FP64 matrix");
  gemv_tree_impl<double, double>(A, nv, alpha, xt, ldx, beta, yt, ldy, s, nt_force);
}

void gemv_tree_f32(const h2_matrix* A, int nv, float alpha, const float* xt, int ldx, float beta,
                   float* yt, int ldy, hipStream_t s, int nt_force) {
  if (nv <= 0) return;
  switch (A->st.prec) {
    case H2_FP64: gemv_tree_impl<double, float>(A, nv, alpha, xt, ldx, beta, yt, ldy, s, nt_force); break;
    case H2_FP32: gemv_tree_impl<float, float>(A, nv, alpha, xt, ldx, beta, yt, ldy, s, nt_force); break;
    case H2_BF16: gemv_tree_impl<bf16_t, float>(A, nv, alpha, xt, ldx, beta, yt, ldy, s, nt_force); break;
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

// ------------------------------------------------------------------ no-allocation product
namespace h2 {

// Workspace of h2_gemv_noalloc: tree-order x and y (n * nv words each) and
// the coefficient vectors (2 * sum of ranks * nv words).  One copy per GPU,
// held until the process ends; every call on a GPU shares it.
constexpr int64_t NOALLOC_WORDS = (int64_t)1 << 23;   // 64 MiB of FP64
static __device__ __align__(256) double scratch[NOALLOC_WORDS];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the array's name is only a host-side stand-in)
double* scratch_ptr() {
  int dev = 0;
  H2_HIP(hipGetDevice(&dev));
  H2_CHECK(dev >= 0 && dev < NOALLOC_MAX_DEVICES, H2_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    H2_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    H2_CHECK(p != nullptr, H2_EDEVICE, "no device address for the workspace array");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

h2_status guarded_status(const std::function<void()>& f);

int64_t gemv_noalloc_words(const h2_matrix* A, int nv) {
  return 2 * ((int64_t)A->tree->n + A->kpre.back()) * (int64_t)nv;
}

}  // namespace h2

using namespace h2;

extern "C" int h2_test_gemv_split_groups(const h2_matrix* A, int nv) {
  if (!A || nv <= 0 || A->tree->L < 1) return 1;
  const int64_t nc = A->tree->nclusters() - 1;
  return split_groups(nc * ((nv + 15) / 16), (double)A->kpre.back() / nc);
}

extern "C" h2_status h2_gemv_noalloc(const h2_matrix* A, int nv, double alpha, const double* x,
                                     int ldx, double beta, double* y, int ldy, hipStream_t s) {
  return guarded_status([&] {
    H2_CHECK(A, H2_EINVAL, "null matrix");
    const h2_tree* t = A->tree;
    const int n = t->n;
    H2_CHECK(nv >= 0 && ldx >= n && ldy >= n, H2_EINVAL, "bad vector count or leading dimension");
    if (nv == 0) return;
    H2_CHECK(x && y, H2_EINVAL, "null vector");
    H2_CHECK(A->st.prec == H2_FP64, H2_EINVAL, "h2_gemv_noalloc needs FP64 storage");
    H2_CHECK(t->device_ready, H2_EINVAL, "tree has no device index arrays");
    H2_CHECK(gemv_noalloc_words(A, nv) <= NOALLOC_WORDS, H2_EINVAL,
             "h2_gemv_noalloc: 2 (n + sum of ranks) nv exceeds the 2^23-word workspace");
    double* ws = scratch_ptr();
    double* xt = ws;
    double* yt = xt + (size_t)n * nv;
    double* coef = yt + (size_t)n * nv;
    // tile width: the autotuned one if this tree has it, else the rule the
    // tuner falls back to (no timing run: it would allocate)
    int nt = 0;
    if (A->kmax <= LEAF_MAX) {
      const std::tuple<int, int, int> key{std::min((nv + 15) / 16, 4), 8, 8};
      auto it = t->tuned_nt.find(key);
      nt = it != t->tuned_nt.end() ? it->second : (nv <= 16 ? 1 : (nv <= 32 ? 2 : 4));
    }
    gather_rows(t, nv, x, ldx, xt, n, s);
    gemv_tree_run<double, double>(A, nv, 1.0, xt, n, 0.0, yt, n, s, nt, coef);
    scatter_rows(t, nv, alpha, yt, n, beta, y, ldy, s);
  });
}
