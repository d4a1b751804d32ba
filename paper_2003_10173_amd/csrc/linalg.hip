// Batched FP64 dense kernels for the construction (Sec. 3.3: sampling by
// batched products, compression by batched QR and SVD).  One launch covers
// every block of a level; descriptors travel in the kernel arguments (small
// batches) or through a pinned staging ring.
//
// The GEMM is a 64x64-tile FP64 FMA kernel (FP64 vector and matrix peaks are
// equal on CDNA4, so the vector path loses nothing for FP64); tall reductions
// (K >> M, N) are split over K into partial tiles that a second kernel sums in
// a fixed order, so results are deterministic.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include <hip/hip_cooperative_groups.h>

#include "kernels_common.h"
#include "linalg.h"
#include "timing.h"

namespace h2 {

// ------------------------------------------------------------------ staging
Staging::Staging(size_t cap_bytes) : cap(cap_bytes) {
  H2_HIP(hipHostMalloc((void**)&host, cap, hipHostMallocDefault));
  dev.alloc(cap);
}
Staging::~Staging() {
  reset();
  if (host) (void)hipHostFree(host);
}
void* Staging::put(const void* src, size_t bytes, hipStream_t s) {
  const size_t n = (bytes + 255) & ~(size_t)255;
  if (head + n > cap) {
    // Continue in a fresh ring: regions handed out since the last reset() may
    // still be read by queued copies and kernels (a launch often takes several
    // arrays), so the old ring stays allocated until reset().
    retired_host.push_back(host);
    retired_dev.push_back(std::move(dev));
    host = nullptr;
    cap = std::max(cap, 2 * n);
    H2_HIP(hipHostMalloc((void**)&host, cap, hipHostMallocDefault));
    dev.alloc(cap);
    head = 0;
  }
  std::memcpy(host + head, src, bytes);
  char* d = dev.as<char>() + head;
  H2_HIP(hipMemcpyAsync(d, host + head, bytes, hipMemcpyHostToDevice, s));
  head += n;
  return d;
}

void Staging::reset() {
  head = 0;
  for (char* h : retired_host)
    if (h) (void)hipHostFree(h);
  retired_host.clear();
  retired_dev.clear();
}

double* Scratch::get(size_t elems) {
  const size_t bytes = ((std::max<size_t>(elems, 1) * sizeof(double)) + 255) & ~(size_t)255;
  if (bufs.empty() || used + bytes > bufs.back().bytes) {
    bufs.emplace_back(std::max(bytes, (size_t)64 << 20));
    used = 0;
  }
  double* p = (double*)(bufs.back().as<char>() + used);
  used += bytes;
  return p;
}

void Scratch::clear() {
  // callers clear only when the stream is idle; merge growth into one buffer
  if (bufs.size() > 1) {
    size_t tot = 0;
    for (auto& b : bufs) tot += b.bytes;
    bufs.clear();
    bufs.emplace_back(tot);
  }
  used = 0;
}

// ------------------------------------------------------------------ descriptor transport
// The descriptor array of a launch travels in its kernel arguments when it is
// small: it is then part of the launch packet, with no copy of its own on the
// stream.  Larger arrays go through the staging ring.  Kernels index both
// forms alike.
template <class T>
struct DevArr {
  const T* p;
  __device__ const T& operator[](int64_t i) const { return p[i]; }
};
template <class T, int N>
struct ArgArr {
  T v[N];
  __device__ const T& operator[](int64_t i) const { return v[i]; }
};
constexpr size_t KARG_MAX = 3072;  // bytes of descriptors per launch's arguments

// launch(arr) with the n descriptors at v as an ArgArr<T, N> (n <= N) or a DevArr<T>
template <int N, class T, class F>
void with_descs(Ctx& c, const T* v, size_t n, F&& launch) {
  static_assert(sizeof(ArgArr<T, N>) <= KARG_MAX, "inline descriptors exceed the argument budget");
  if (n <= (size_t)N) {
    ArgArr<T, N> a{};
    std::memcpy(a.v, v, n * sizeof(T));
    launch(a);
  } else {
    launch(DevArr<T>{(const T*)c.stage.put(v, n * sizeof(T), c.s)});
  }
}

// ------------------------------------------------------------------ GEMM
constexpr int TM = 64, TN = 64, TK = 32, TQ = TM * TK / 256;

struct GemmTask {
  GemmDesc d;
  int tiles_m, tiles_n;
  int k0, k1;           // K range of this task
  double* out;          // output (C or a partial buffer)
  int ldo;
  double beta;          // applied to `out`
};

// One 64 x 64 output tile per workgroup.  The K range is walked in blocks
// of TK: every block is read from memory into registers one block ahead of
// its use (clamped, in-range addresses; the positions outside the operands
// are zeroed when stored), stored into one of two LDS tile buffers and
// multiplied there on the matrix cores after a single barrier, so that the
// loads of the next block overlap the products of this one.
template <class TA, class SA>
__global__ __launch_bounds__(256) void k_gemm(TA tasks, SA tile_start, int ntasks) {
  __shared__ double As[2][TK][TM + 1];
  __shared__ double Bs[2][TK][TN + 1];
  // locate the task of this block
  int lo = 0, hi = ntasks - 1;
  const int64_t b = blockIdx.x;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const GemmTask& t = tasks[lo];
  const GemmDesc& d = t.d;
  if (d.run && *d.run == 0) return;
  const int tile = (int)(b - tile_start[lo]);
  const int bm = (tile % t.tiles_m) * TM, bn = (tile / t.tiles_m) * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // wave w: rows 32 (w % 2) .. +32, columns 32 (w / 2) .. +32 of the tile, as
  // 2 x 2 sub-tiles of 16 x 16 on the FP64 matrix cores (16x16x4 products)
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int wr = 32 * (wave & 1), wc = 32 * (wave >> 1);
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  // this thread's elements of a block: A (i, k) and B (k, j) for q < TQ
  // (consecutive threads along the operand's contiguous dimension)
  int ai[TQ], ak[TQ], bj[TQ], bk[TQ];
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    const int e = tid + 256 * q;
    if (!d.ta) { ai[q] = e % TM; ak[q] = e / TM; } else { ak[q] = e % TK; ai[q] = e / TK; }
    if (!d.tb) { bk[q] = e % TK; bj[q] = e / TK; } else { bj[q] = e % TN; bk[q] = e / TN; }
  }
  const int mc = d.M - 1, nc = d.N - 1;
  // (global-memory pointers: their loads count only against the vector
  // memory counter, not against the LDS one that the tile reads wait on)
  typedef const double __attribute__((address_space(1)))* gptr;
  const gptr Ag = (gptr)d.A, Bg = (gptr)d.B;
  double va[TQ], vb[TQ];
  auto gload = [&](int k0) {
    const int kl = t.k1 - 1;
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const int gi = min(bm + ai[q], mc), gk = min(k0 + ak[q], kl);
      va[q] = d.ta ? Ag[(size_t)gi * d.lda + gk] : Ag[(size_t)gk * d.lda + gi];
      const int gj = min(bn + bj[q], nc), gk2 = min(k0 + bk[q], kl);
      vb[q] = d.tb ? Bg[(size_t)gk2 * d.ldb + gj] : Bg[(size_t)gj * d.ldb + gk2];
    }
  };
  auto lstore = [&](int k0, int buf) {
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      As[buf][ak[q]][ai[q]] = (bm + ai[q] < d.M && k0 + ak[q] < t.k1) ? va[q] : 0.0;
      Bs[buf][bk[q]][bj[q]] = (bn + bj[q] < d.N && k0 + bk[q] < t.k1) ? vb[q] : 0.0;
    }
  };
  if (t.k0 < t.k1) gload(t.k0);
  int buf = 0;
  for (int k0 = t.k0; k0 < t.k1; k0 += TK) {
    // buffer buf was last read by the products of block k0 - 2 TK, which
    // every wave finished before the barrier of block k0 - TK
    lstore(k0, buf);
    __syncthreads();
    if (k0 + TK < t.k1) gload(k0 + TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kk = ks + (lane >> 4);
      double a[2], bb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[buf][kk][wr + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bb[j] = Bs[buf][kk][wc + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    buf ^= 1;
  }
  // result register r of a 16 x 16 f64 product: row 4 r + lane / 16, column
  // lane % 16; with beta != 0 the 16 old values are read first, together
  typedef double __attribute__((address_space(1)))* gout;
  const gout Og = (gout)t.out;
  double old[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = bm + wr + 16 * i + 4 * r + (lane >> 4);
        const int gj = bn + wc + 16 * j + (lane & 15);
        old[i][j][r] = (t.beta != 0.0 && gi < d.M && gj < d.N) ? Og[(size_t)gj * t.ldo + gi] : 0.0;
      }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = bm + wr + 16 * i + 4 * r + (lane >> 4);
        const int gj = bn + wc + 16 * j + (lane & 15);
        if (gi < d.M && gj < d.N) {
          const double v = d.alpha * acc[i][j][r];
          Og[(size_t)gj * t.ldo + gi] = t.beta == 0.0 ? v : v + t.beta * old[i][j][r];
        }
      }
}

struct ReduceTask {
  double* C;
  int ldc, M, N;
  double beta;
  const double* parts;  // nparts consecutive M x N blocks (ld = M)
  int nparts;
  const int* run;       // optional: skipped when *run == 0
};

template <class RA>
__global__ void k_reduce_parts(RA tasks, int ntasks) {
  const ReduceTask& t = tasks[blockIdx.y];
  if (t.run && *t.run == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)t.M * t.N) return;
  const int i = (int)(e % t.M), j = (int)(e / t.M);
  double s = 0;
  for (int p = 0; p < t.nparts; ++p) s += t.parts[(size_t)p * t.M * t.N + e];
  double* o = t.C + (size_t)j * t.ldc + i;
  *o = t.beta == 0.0 ? s : s + t.beta * *o;
}

constexpr int GEMM_ARG_TASKS = 20;
static_assert(sizeof(ArgArr<GemmTask, GEMM_ARG_TASKS>) + sizeof(ArgArr<int64_t, GEMM_ARG_TASKS + 1>) <= KARG_MAX,
              "GEMM tasks exceed the argument budget");

void gemm_batched(Ctx& c, const std::vector<GemmDesc>& ds) {
  std::vector<GemmTask> tasks;
  std::vector<ReduceTask> reds;
  constexpr int KMIN = 128;
  for (const auto& d : ds) {
    if (d.M <= 0 || d.N <= 0) continue;
    const int tm = (d.M + TM - 1) / TM, tn = (d.N + TN - 1) / TN;
    if (d.K <= 0) {
      // C = beta C only
      GemmTask t{d, tm, tn, 0, 0, d.C, d.ldc, d.beta};
      tasks.push_back(t);
      continue;
    }
    // split K for products with few output tiles (the K loop is serial per
    // tile): chunks of at least KMIN, about 128 tiles in all, decided per
    // product alone so that a product's sums do not depend on its batch
    int nsplit = 1;
    if (d.K >= 2 * KMIN && tm * tn < 128)
      nsplit = std::max(1, std::min({64, d.K / KMIN, (128 + tm * tn - 1) / (tm * tn)}));
    if (nsplit == 1) {
      tasks.push_back(GemmTask{d, tm, tn, 0, d.K, d.C, d.ldc, d.beta});
    } else {
      double* parts = c.scratch.get((size_t)nsplit * d.M * d.N);
      const int chunk = ((d.K + nsplit - 1) / nsplit + TK - 1) / TK * TK;
      int used = 0;
      for (int p = 0; p < nsplit; ++p) {
        const int k0 = p * chunk, k1 = std::min(d.K, k0 + chunk);
        if (k0 >= k1) break;
        tasks.push_back(GemmTask{d, tm, tn, k0, k1, parts + (size_t)p * d.M * d.N, d.M, 0.0});
        ++used;
      }
      reds.push_back(ReduceTask{d.C, d.ldc, d.M, d.N, d.beta, parts, used, d.run});
    }
  }
  if (tasks.empty()) return;
  std::vector<int64_t> start(tasks.size() + 1, 0);
  for (size_t i = 0; i < tasks.size(); ++i)
    start[i + 1] = start[i] + (int64_t)tasks[i].tiles_m * tasks[i].tiles_n;
  H2_CHECK(start.back() < (int64_t)1 << 31, H2_EINVAL, "GEMM batch too large");
  const unsigned nblk = (unsigned)start.back();
  if (tasks.size() <= GEMM_ARG_TASKS) {
    // tasks and tile offsets in the kernel arguments
    ArgArr<GemmTask, GEMM_ARG_TASKS> ta{};
    ArgArr<int64_t, GEMM_ARG_TASKS + 1> sa{};
    std::memcpy(ta.v, tasks.data(), tasks.size() * sizeof(GemmTask));
    std::memcpy(sa.v, start.data(), start.size() * sizeof(int64_t));
    k_gemm<<<nblk, 256, 0, c.s>>>(ta, sa, (int)tasks.size());
  } else {
    // tasks and tile offsets in one upload
    const size_t bt = tasks.size() * sizeof(GemmTask), bs = start.size() * sizeof(int64_t);
    const size_t os = (bt + 15) & ~(size_t)15;
    std::vector<char> blob(os + bs);
    std::memcpy(blob.data(), tasks.data(), bt);
    std::memcpy(blob.data() + os, start.data(), bs);
    char* dblob = (char*)c.stage.put(blob.data(), blob.size(), c.s);
    k_gemm<<<nblk, 256, 0, c.s>>>(DevArr<GemmTask>{(const GemmTask*)dblob},
                                  DevArr<int64_t>{(const int64_t*)(dblob + os)}, (int)tasks.size());
  }
  H2_LAUNCH_CHECK();
  if (!reds.empty()) {
    int64_t mx = 0;
    for (auto& r : reds) mx = std::max(mx, (int64_t)r.M * r.N);
    for (size_t i0 = 0; i0 < reds.size(); i0 += 65535) {
      const size_t cnt = std::min<size_t>(65535, reds.size() - i0);
      dim3 grid((unsigned)((mx + 255) / 256), (unsigned)cnt);
      with_descs<32>(c, reds.data() + i0, cnt, [&](auto ra) {
        k_reduce_parts<<<grid, 256, 0, c.s>>>(ra, (int)cnt);
      });
      H2_LAUNCH_CHECK();
    }
  }
}

// ------------------------------------------------------------------ Householder QR
constexpr int QR_VCACHE = 8192;

// stream-ordered timing of a section, active only with verbose output
struct VTimer {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t s;
  explicit VTimer(hipStream_t st) : s(st) {
    if (!verbose()) return;
    H2_HIP(hipEventCreate(&e0));
    H2_HIP(hipEventCreate(&e1));
    H2_HIP(hipEventRecord(e0, s));
  }
  bool on() const { return e0 != nullptr; }
  float stop() {
    float ms = 0;
    H2_HIP(hipEventRecord(e1, s));
    H2_HIP(hipEventSynchronize(e1));
    H2_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms;
  }
  ~VTimer() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};  // rows of the current reflector kept in LDS

__global__ __launch_bounds__(256) void k_qr(const QRDesc* __restrict__ descs) {
  const QRDesc d = descs[blockIdx.x];
  __shared__ double vcache[QR_VCACHE];
  __shared__ double taus[1024];
  __shared__ double red[8];
  __shared__ double bcast[2];
  const int m = d.m, n = d.n, kmin = min(m, n);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* A = d.A;
  const int lda = d.lda;
  for (int j = 0; j < kmin; ++j) {
    double* aj = A + (size_t)j * lda;
    double s = 0;
    for (int i = j + 1 + tid; i < m; i += 256) s += aj[i] * aj[i];
    s = block_sum256(s, red);
    if (tid == 0) {
      const double alpha = aj[j];
      double tau = 0, scale = 0;
      if (s != 0.0) {
        const double norm = sqrt(alpha * alpha + s);
        const double beta = alpha >= 0 ? -norm : norm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
        aj[j] = beta;
      }
      bcast[0] = tau;
      bcast[1] = scale;
      taus[j] = tau;
    }
    __syncthreads();
    const double tau = bcast[0], scale = bcast[1];
    const bool cached = (m - j) <= QR_VCACHE;
    for (int i = j + 1 + tid; i < m; i += 256) {
      const double v = aj[i] * scale;
      aj[i] = v;
      if (cached) vcache[i - j] = v;
    }
    if (tid == 0 && cached) vcache[0] = 1.0;
    __syncthreads();
    if (tau != 0.0) {
      for (int col = j + 1 + wave; col < n; col += 4) {
        double* ac = A + (size_t)col * lda;
        double w = 0;
        for (int i = j + lane; i < m; i += 64) {
          const double v = i == j ? 1.0 : (cached ? vcache[i - j] : aj[i]);
          w += v * ac[i];
        }
        w = wave_sum(w) * tau;
        for (int i = j + lane; i < m; i += 64) {
          const double v = i == j ? 1.0 : (cached ? vcache[i - j] : aj[i]);
          ac[i] -= v * w;
        }
      }
    }
    __syncthreads();
  }
  // R (kmin x n, upper trapezoidal)
  if (d.R) {
    for (int e = tid; e < kmin * n; e += 256) {
      const int i = e % kmin, c = e / kmin;
      d.R[(size_t)c * d.ldr + i] = i <= c ? A[(size_t)c * lda + i] : 0.0;
    }
  }
  if (!d.Q) return;
  // explicit thin Q = H_0 ... H_{kmin-1} [I; 0]
  for (int e = tid; e < m * kmin; e += 256) {
    const int i = e % m, c = e / m;
    d.Q[(size_t)c * d.ldq + i] = i == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = kmin - 1; j >= 0; --j) {
    const double tau = taus[j];
    if (tau == 0.0) continue;
    const double* aj = A + (size_t)j * lda;
    const bool cached = (m - j) <= QR_VCACHE;
    if (cached) {
      for (int i = j + 1 + tid; i < m; i += 256) vcache[i - j] = aj[i];
      if (tid == 0) vcache[0] = 1.0;
    }
    __syncthreads();
    for (int col = j + wave; col < kmin; col += 4) {
      double* qc = d.Q + (size_t)col * d.ldq;
      double w = 0;
      for (int i = j + lane; i < m; i += 64) {
        const double v = i == j ? 1.0 : (cached ? vcache[i - j] : aj[i]);
        w += v * qc[i];
      }
      w = wave_sum(w) * tau;
      for (int i = j + lane; i < m; i += 64) {
        const double v = i == j ? 1.0 : (cached ? vcache[i - j] : aj[i]);
        qc[i] -= v * w;
      }
    }
    __syncthreads();
  }
}

void qr_batched(Ctx& c, const std::vector<QRDesc>& ds) {
  std::vector<QRDesc> v;
  for (auto& d : ds) {
    if (d.m <= 0 || d.n <= 0) continue;
    H2_CHECK(std::min(d.m, d.n) <= 1024, H2_EINVAL, "QR: more than 1024 columns");
    v.push_back(d);
  }
  if (v.empty()) return;
  auto* dd = (QRDesc*)c.stage.put(v.data(), v.size() * sizeof(QRDesc), c.s);
  k_qr<<<(unsigned)v.size(), 256, 0, c.s>>>(dd);
  H2_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ Jacobi SVD
// One-sided (Hestenes) Jacobi: columns a, b of A (m rows) are rotated until
// every pair is orthogonal to 1e-15 relative; V accumulates the rotations.
// Pairs follow the round-robin tournament (np = n rounded up to even; np - 1
// rounds per sweep, np / 2 disjoint pairs per round).
__device__ inline void tournament_pair(int np, int r, int k, int& a, int& b) {
  if (k == 0) { a = np - 1; b = r; }
  else { a = (r + k) % (np - 1); b = (r - k + (np - 1)) % (np - 1); }
  if (a > b) { const int t = a; a = b; b = t; }
}

// Rotation threshold: columns count as orthogonal once |a.b| <= tol |a| |b|
// with tol at the rounding level of an m-term dot product, so that no sweep
// is spent on rotations that only move rounding noise around.
__device__ inline double jacobi_tol(int m) { return fmax(1e-15, (double)m * 0x1p-53); }

// rotate columns a < b of A (and V) by one wave; returns true if rotated
__device__ inline bool jacobi_rotate(double* A, int lda, int m, double* V, int ldv, int n, int a,
                                     int b, int lane, double tol) {
  double* ca = A + (size_t)a * lda;
  double* cb = A + (size_t)b * lda;
  double al = 0, be = 0, ga = 0;
  for (int i = lane; i < m; i += 64) {
    const double x = ca[i], y = cb[i];
    al += x * x;
    be += y * y;
    ga += x * y;
  }
  double sums[3] = {al, be, ga};
  wave_sum_n(sums);
  al = sums[0];
  be = sums[1];
  ga = sums[2];
  if (ga == 0.0 || !(fabs(ga) > tol * sqrt(al) * sqrt(be))) return false;
  const double zeta = (be - al) / (2.0 * ga);
  double t;
  if (fabs(zeta) > 1e150) t = 0.5 / zeta;
  else t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
  for (int i = lane; i < m; i += 64) {
    const double x = ca[i], y = cb[i];
    ca[i] = cs * x - sn * y;
    cb[i] = sn * x + cs * y;
  }
  if (V) {
    double* va = V + (size_t)a * ldv;
    double* vb = V + (size_t)b * ldv;
    for (int i = lane; i < n; i += 64) {
      const double x = va[i], y = vb[i];
      va[i] = cs * x - sn * y;
      vb[i] = sn * x + cs * y;
    }
  }
  return true;
}

// V = I, a workgroup per 16 columns (blockIdx.y)
__global__ void k_svd_init_v(const SVDDesc* __restrict__ descs) {
  const SVDDesc d = descs[blockIdx.x];
  if (!d.V) return;
  const int c0 = 16 * blockIdx.y;
  for (int c = c0; c < min(d.n, c0 + 16); ++c)
    for (int i = threadIdx.x; i < d.n; i += blockDim.x) d.V[(size_t)c * d.ldv + i] = i == c ? 1.0 : 0.0;
}

// single workgroup per matrix (small n): 8 waves rotate 8 disjoint pairs at a time
__global__ __launch_bounds__(512) void k_svd_sweeps(const SVDDesc* __restrict__ descs) {
  const SVDDesc d = descs[blockIdx.x];
  const int n = d.n, m = d.m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ int rotated;
  const int np = n + (n & 1);
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      for (int k = wave; k < np / 2; k += 8) {
        int a, b;
        tournament_pair(np, r, k, a, b);
        if (b >= n) continue;
        if (jacobi_rotate(d.A, d.lda, m, d.V, d.ldv, n, a, b, lane, fmax(d.tol, jacobi_tol(m))) &&
            lane == 0)
          rotated = 1;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
}

// Block one-sided Jacobi over many workgroups: columns are grouped in blocks
// of SVD_BS; each round of the block tournament gives every workgroup one
// pair of blocks.  Its 2*SVD_BS columns are staged in LDS, their Gram matrix
// G = L^T L is formed on the FP64 matrix cores, and the small symmetric
// problem G = W diag W^T is solved by cyclic two-sided Jacobi on G (parallel
// tournament order, one wave, up to SVD_INNER sweeps); the columns of A and
// of V are then multiplied by the accumulated rotation W once.  Whether a
// pair still needs rotating is decided on the Gram matrix of the current
// columns (|a.b| > tol |a| |b|), so a sweep without rotations certifies the
// columns themselves.  Rounds are ordered by data flow: each block carries the
// number of rounds it has been through, and a workgroup starts a round once
// both of its blocks have finished the previous one (release/acquire at
// device scope).  One grid-wide barrier per sweep precedes the termination
// test, which every workgroup takes from the same flags.  A wait that does not
// end within a few seconds marks status[1] (the singular values of the call
// then come out as NaN) instead of hanging.
constexpr int SVD_BS = 8, SVD_PC = 2 * SVD_BS, SVD_MMAX = 1024, SVD_INNER = 1, SVD_VPF = 4;
static_assert((SVD_BS & (SVD_BS - 1)) == 0, "the cross-pair steps index blocks by masking");
typedef double svd_d4 __attribute__((ext_vector_type(4)));

// the pairs of tournament_pair without integer division (r < np - 1, k < np / 2)
__device__ inline void tournament_pair_fast(int np, int r, int k, int& a, int& b) {
  if (k == 0) { a = np - 1; b = r; }
  else {
    a = r + k;
    if (a >= np - 1) a -= np - 1;
    b = r - k;
    if (b < 0) b += np - 1;
  }
  if (a > b) { const int t = a; a = b; b = t; }
}

// columns a, b (Gram entries al = a.a, be = b.b, ga = a.b) need a rotation
__device__ inline bool jacobi_needs(double al, double be, double ga, double tol) {
  return ga != 0.0 && ga * ga > (tol * tol) * (al * be);
}

// rotation a <- c a - s b, b <- s a + c b that makes a.b vanish:
// t = sign(d e) |e| / (|d| + sqrt(d^2 + e^2)) with d = be - al, e = 2 ga is the
// smaller root of t^2 + 2 (d / e) t - 1 = 0; c = 1 / sqrt(1 + t^2), s = c t
__device__ inline void jacobi_cs(double al, double be, double ga, double& c, double& s) {
  const double d = be - al, e = 2.0 * ga;
  const double h = sqrt(d * d + e * e);
  double t = fabs(e) / (fabs(d) + h);
  if ((d < 0) != (e < 0) && d != 0.0) t = -t;
  c = rsqrt(1.0 + t * t);
  s = c * t;
}

// wait until *p >= v (device-scope load); false after `limit` polls (the
// default, SVD_SPIN, is a few seconds)
constexpr int SVD_SPIN = 1 << 22;
__device__ inline bool svd_wait(const int* p, int v, int limit) {
  for (int it = 0; it < limit; ++it) {
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= v) return true;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

// LDS ordering between the lanes of one wave (the wave runs in lockstep):
// every LDS access issued before has completed, and no access is moved
// across by the compiler
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// flags: 3 x nmat rotation flags (one set per sweep, in turn); ver: nmat x
// maxnb round counters of the blocks; status[0] = sweeps, status[1] = wait
// timeout (all zero at launch)
__global__ __launch_bounds__(512) void k_svd_block(const SVDDesc* __restrict__ descs,
                                                   const int* __restrict__ wg_start, int nmat,
                                                   int maxnb, int* flags, int* ver, int* status,
                                                   int spin) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  __shared__ double L[SVD_PC * SVD_MMAX];
  __shared__ double Gp[8 * SVD_PC * SVD_PC];      // per-wave Gram partials
  __shared__ double Gs[SVD_PC * SVD_PC];          // Gram, G(i, j) at [i * 16 + j]
  __shared__ double Ws[SVD_PC * SVD_PC];          // rotation, W(q, j) at [q * 16 + j]
  __shared__ int cols[SVD_PC];
  __shared__ int rot_any;
  int lo = 0, hi = nmat - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wg_start[mid] <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const int mi = lo;
  const SVDDesc d = descs[mi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwg = wg_start[mi + 1] - wg_start[mi];
  const int wl = (int)blockIdx.x - wg_start[mi];
  const int n = d.n, m = d.m;
  const int nb = (n + SVD_BS - 1) / SVD_BS;
  const int npb = nb + (nb & 1);
  const double tol = fmax(d.tol, jacobi_tol(m));
  int* vb = ver + (size_t)mi * maxnb;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int* fl = flags + (sweep % 3) * nmat;
    // the set used two sweeps ago is free again: clear it for the next sweep
    if (blockIdx.x == 0 && tid == 0)
      for (int i = 0; i < nmat; ++i) atomicExch(&flags[((sweep + 1) % 3) * nmat + i], 0);
    for (int r = 0; r < npb - 1; ++r) {
      for (int k = wl; k < npb / 2; k += nwg) {
        int bi, bj;
        tournament_pair(npb, r, k, bi, bj);
        const int rq = sweep * (npb - 1) + r;   // rounds both blocks went through before
        // gather the columns of both blocks (the dummy block has none)
        if (tid == 0) {
          bool ok = true;
          if (bi < nb) ok = svd_wait(vb + bi, rq, spin) && ok;
          if (bj < nb) ok = svd_wait(vb + bj, rq, spin) && ok;
          if (!ok) atomicOr(status + 1, 1);
          __threadfence();
          int c = 0;
          for (int q = 0; q < SVD_BS; ++q) {
            const int ci = bi * SVD_BS + q;
            if (bi < nb && ci < n) cols[c++] = ci;
          }
          for (int q = 0; q < SVD_BS; ++q) {
            const int cj = bj * SVD_BS + q;
            if (bj < nb && cj < n) cols[c++] = cj;
          }
          for (; c < SVD_PC; ++c) cols[c] = -1;
          rot_any = 0;
        }
        __syncthreads();
        int nc = 0;
        for (int q = 0; q < SVD_PC; ++q) nc += cols[q] >= 0;
        // the first SVD_VPF row tiles of V this wave updates at the end of the
        // round, loaded now so that their latency overlaps the work below
        // (layout of the matrix-core operand used there)
        double vpf[SVD_VPF][4];
#pragma unroll
        for (int t = 0; t < SVD_VPF; ++t) {
          const int ar = 16 * (wave + 8 * t) + (lane & 15);
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int q = 4 * kk + (lane >> 4);
            vpf[t][kk] = (d.V && q < nc && ar < n) ? d.V[(size_t)cols[q] * d.ldv + ar] : 0.0;
          }
        }
        {
          // all loads of the pair's columns issued before any is stored
          constexpr int RS = SVD_MMAX / 512;
          double xv[SVD_PC][RS];
#pragma unroll
          for (int q = 0; q < SVD_PC; ++q) {
            const double* col = q < nc ? d.A + (size_t)cols[q] * d.lda : nullptr;
#pragma unroll
            for (int sr = 0; sr < RS; ++sr) {
              const int row = tid + 512 * sr;
              xv[q][sr] = (col && row < m) ? col[row] : 0.0;
            }
          }
#pragma unroll
          for (int q = 0; q < SVD_PC; ++q)
#pragma unroll
            for (int sr = 0; sr < RS; ++sr) {
              const int row = tid + 512 * sr;
              if (row < m) L[q * m + row] = xv[q][sr];
            }
        }
        __syncthreads();
        // Gram partials on the matrix cores: wave w takes rows 4 kb .. 4 kb + 3
        // for kb = w, w + 8, ...; lane l supplies L(row 4 kb + l / 16, column
        // l % 16) as both operands; result element (4 e + l / 16, l % 16) in acc[e]
        // (four k-blocks per step: their LDS reads are issued together and
        // feed two accumulators, so neither waits on the other)
        {
          svd_d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
          const int col = lane & 15, kr = lane >> 4;
          const bool cok = col < nc;
          for (int kb = wave; 4 * kb < m; kb += 32) {
            double x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int row = 4 * (kb + 8 * u) + kr;
              x[u] = (row < m && cok) ? L[col * m + row] : 0.0;
            }
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[0], x[0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[1], x[1], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[2], x[2], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[3], x[3], acc1, 0, 0, 0);
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) Gp[wave * 256 + (4 * e + kr) * SVD_PC + col] = acc0[e] + acc1[e];
        }
        __syncthreads();
        if (tid < SVD_PC * SVD_PC) {
          double g = 0;
#pragma unroll
          for (int w = 0; w < 8; ++w) g += Gp[w * 256 + tid];
          Gs[tid] = g;
          Ws[tid] = (tid / SVD_PC == tid % SVD_PC) ? 1.0 : 0.0;
        }
        __syncthreads();
        // Pairs of columns from the two blocks meet in every round; pairs
        // within one block need one visit per sweep, which they get in the
        // sweep's first round (and in any round with a partial block).  The
        // other rounds test and rotate only the cross pairs.
        const bool full = r == 0 || nc < SVD_PC;
        // convergence test on the Gram matrix of the current columns
        if (tid < SVD_PC * SVD_PC) {
          const int i = tid / SVD_PC, j = tid % SVD_PC;
          if (i < j && j < nc && (full || (i < SVD_BS && j >= SVD_BS))) {
            if (jacobi_needs(Gs[i * 17], Gs[j * 17], Gs[tid], tol)) rot_any = 1;
          }
        }
        __syncthreads();
        if (rot_any && wave == 0) {
          // cyclic two-sided Jacobi on G, W accumulating the rotations.  In
          // each step lane (P, Q) = (lane / 8, lane % 8) owns the 2 x 2 block of
          // G and of W at rows of pair P and columns of pair Q, so the update
          // G <- J^T G J, W <- W J stays within the lane
          double* G = Gs;
          double* Wm = Ws;
          const int npc = nc + (nc & 1);
          const int P = lane >> 3, Q = lane & 7;
          const bool act = P < npc / 2 && Q < npc / 2;
          // full rounds: the tournament over all 2 SVD_BS columns; otherwise
          // the SVD_BS steps that pair column P of the first block with
          // column (P + step) mod SVD_BS of the second
          const int nsteps = full ? npc - 1 : SVD_BS;
          for (int isw = 0; isw < SVD_INNER; ++isw) {
            int rotated = 0;
            for (int rr = 0; rr < nsteps; ++rr) {
              int aP = 0, bP = 0, aQ = 0, bQ = 0;
              double g00 = 0, g01 = 0, g10 = 0, g11 = 0, w00 = 0, w01 = 0, w10 = 0, w11 = 0;
              double pa = 0, pb = 0, pg = 0, qa = 0, qb = 0, qg = 0;
              if (act) {
                if (full) {
                  tournament_pair_fast(npc, rr, P, aP, bP);
                  tournament_pair_fast(npc, rr, Q, aQ, bQ);
                } else {
                  aP = P;
                  bP = SVD_BS + ((P + rr) & (SVD_BS - 1));
                  aQ = Q;
                  bQ = SVD_BS + ((Q + rr) & (SVD_BS - 1));
                }
                g00 = G[aP * SVD_PC + aQ];
                g01 = G[aP * SVD_PC + bQ];
                g10 = G[bP * SVD_PC + aQ];
                g11 = G[bP * SVD_PC + bQ];
                w00 = Wm[aP * SVD_PC + aQ];
                w01 = Wm[aP * SVD_PC + bQ];
                w10 = Wm[bP * SVD_PC + aQ];
                w11 = Wm[bP * SVD_PC + bQ];
                pa = G[aP * 17];
                pb = G[bP * 17];
                pg = G[aP * SVD_PC + bP];
                qa = G[aQ * 17];
                qb = G[bQ * 17];
                qg = G[aQ * SVD_PC + bQ];
              }
              // every lane forms the rotations of its two pairs itself
              double cP = 1.0, sP = 0.0, cQ = 1.0, sQ = 0.0;
              if (act && bP < nc && jacobi_needs(pa, pb, pg, tol)) jacobi_cs(pa, pb, pg, cP, sP);
              if (act && bQ < nc && jacobi_needs(qa, qb, qg, tol)) jacobi_cs(qa, qb, qg, cQ, sQ);
              rotated |= __any(sP != 0.0);
              if (act) {
                // J = [[c, s], [-s, c]] on (a, b)
                const double h00 = g00 * cQ - g01 * sQ, h01 = g00 * sQ + g01 * cQ;
                const double h10 = g10 * cQ - g11 * sQ, h11 = g10 * sQ + g11 * cQ;
                G[aP * SVD_PC + aQ] = cP * h00 - sP * h10;
                G[aP * SVD_PC + bQ] = cP * h01 - sP * h11;
                G[bP * SVD_PC + aQ] = sP * h00 + cP * h10;
                G[bP * SVD_PC + bQ] = sP * h01 + cP * h11;
                Wm[aP * SVD_PC + aQ] = w00 * cQ - w01 * sQ;
                Wm[aP * SVD_PC + bQ] = w00 * sQ + w01 * cQ;
                Wm[bP * SVD_PC + aQ] = w10 * cQ - w11 * sQ;
                Wm[bP * SVD_PC + bQ] = w10 * sQ + w11 * cQ;
              }
              wave_lds_sync();
            }
            if (!rotated) break;
          }
        }
        __syncthreads();
        const double* W = Ws;
        // restore the orthogonality of the accumulated rotation lost to
        // rounding (one Newton-Schulz polar step Q <- Q (3I - Q^T Q) / 2) so
        // that the many block products applied to V do not drift
        if (rot_any) {
          double* Gl = Gp;
          double* Wq = Gp + 256;
          if (tid < SVD_PC * SVD_PC) {
            const int i = tid / SVD_PC, j = tid % SVD_PC;
            double g = 0;
            for (int p = 0; p < SVD_PC; ++p) g += W[p * SVD_PC + i] * W[p * SVD_PC + j];
            Gl[tid] = ((i == j ? 3.0 : 0.0) - g) * 0.5;
          }
          __syncthreads();
          if (tid < SVD_PC * SVD_PC) {
            const int q = tid / SVD_PC, j = tid % SVD_PC;
            double acc = 0;
            for (int p = 0; p < SVD_PC; ++p) acc += W[q * SVD_PC + p] * Gl[p * SVD_PC + j];
            Wq[tid] = acc;
          }
          __syncthreads();
        }
        const double* Wf = Gp + 256;
        // columns of A (from LDS) and of V (from memory) times W on the matrix
        // cores, 16 rows per product, formed transposed as W^T X^T: lane l
        // supplies W(k0 + l / 16, l % 16) as the first operand and X(row
        // r0 + l % 16, column k0 + l / 16) as the second; acc[e] then holds
        // (X W)(r0 + l % 16, 4 e + l / 16), so the 16 lanes of one column
        // store 16 consecutive rows
        if (rot_any) {
          const int kr = lane >> 4, cl = lane & 15;
          double wb[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) wb[kk] = Wf[(4 * kk + kr) * SVD_PC + cl];
          // one 16-row tile: X (lane operand x[kk]) times W, stored to Y
          auto tile = [&](const double (&x)[4], double* Y, int ldy, int r0, int rows) {
            svd_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wb[kk], x[kk], acc, 0, 0, 0);
            const int row = r0 + cl;
            if (row < rows) {
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int q = 4 * e + kr;
                if (q < nc) Y[(size_t)cols[q] * ldy + row] = acc[e];
              }
            }
          };
          if (d.V) {
#pragma unroll
            for (int t = 0; t < SVD_VPF; ++t)
              if (16 * (wave + 8 * t) < n) tile(vpf[t], d.V, d.ldv, 16 * (wave + 8 * t), n);
            for (int r0 = 16 * (wave + 8 * SVD_VPF); r0 < n; r0 += 128) {
              double x[4];
#pragma unroll
              for (int kk = 0; kk < 4; ++kk) {
                const int q = 4 * kk + kr;
                x[kk] = (q < nc && r0 + cl < n) ? d.V[(size_t)cols[q] * d.ldv + r0 + cl] : 0.0;
              }
              tile(x, d.V, d.ldv, r0, n);
            }
          }
          for (int r0 = 16 * wave; r0 < m; r0 += 128) {
            double x[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
              const int q = 4 * kk + kr;
              x[kk] = (q < nc && r0 + cl < m) ? L[q * m + r0 + cl] : 0.0;
            }
            tile(x, d.A, d.lda, r0, m);
          }
          if (tid == 0) atomicOr(&fl[mi], 1);
        }
        // both blocks have been through round rq: publish after all writes.
        // The barrier alone does not wait for other waves' global stores
        // (its workgroup-scope fence needs no such wait within one compute
        // unit), so every wave first waits until its own stores of A and V
        // have completed at the L2; thread 0's device-scope release then
        // writes the L2 back, covering every wave's stores, before the
        // counter is published (a workgroup that acquires the counter at
        // device scope reads them from memory)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
          __threadfence();
          if (bi < nb) atomicExch(vb + bi, rq + 1);
          if (bj < nb) atomicExch(vb + bj, rq + 1);
        }
      }
    }
    grid.sync();
    int any = 0;
    for (int i = 0; i < nmat; ++i) any |= atomicAdd(&fl[i], 0);
    if (!any || sweep == 59) {
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(status, sweep + 1);
      break;
    }
  }
}

// ranking key of a singular value: NaN ranks below every number
__device__ inline double svd_rank_key(double s) { return s == s ? s : -__builtin_inf(); }

// singular values = column norms, sorted descending; U = normalised columns;
// V columns permuted alike.  k_svd_order (one workgroup per matrix) finds
// the norms and their order; k_svd_permute and k_svd_vback (a workgroup per
// 16 output columns) write U and the permuted V through a scratch copy.
// status[1] set (a block Jacobi wait timed out): singular values are NaN
struct SvdFin {
  int* ord;      // n: source column of output column r
  double* nrm;   // n: column norms, unsorted
  double* T;     // n x n (ld n): permuted V before it is copied back
};

__global__ __launch_bounds__(1024) void k_svd_order(const SVDDesc* __restrict__ descs,
                                                    const SvdFin* __restrict__ fin,
                                                    const int* __restrict__ status) {
  const SVDDesc d = descs[blockIdx.x];
  const SvdFin f = fin[blockIdx.x];
  const int n = d.n, m = d.m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double sig[1024];
  const double* A = d.A;
  const int lda = d.lda;
  for (int col = wave; col < n; col += 16) {
    const double* ca = A + (size_t)col * lda;
    double s = 0;
    for (int i = lane; i < m; i += 64) s += ca[i] * ca[i];
    s = wave_sum(s);
    if (lane == 0) sig[col] = sqrt(s);
  }
  __syncthreads();
  // descending order, equal values by index: position of i = number of
  // values ranked before it.  A value that is not a number ranks as -inf, so
  // the ranking is a total order and ord a permutation for any input
  const bool failed = status[1] != 0;
  for (int i = tid; i < n; i += 1024) {
    const double si = svd_rank_key(sig[i]);
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double sj = svd_rank_key(sig[j]);
      r += (sj > si) || (sj == si && j < i);
    }
    f.ord[r] = i;
    f.nrm[i] = sig[i];
    d.sigma[r] = failed ? __builtin_nan("") : sig[i];
  }
}

// output columns 16 y .. 16 y + 15 of matrix x: U(:, r) = A(:, ord r) / nrm,
// T(:, r) = V(:, ord r)
__global__ __launch_bounds__(256) void k_svd_permute(const SVDDesc* __restrict__ descs,
                                                     const SvdFin* __restrict__ fin) {
  const SVDDesc d = descs[blockIdx.x];
  const SvdFin f = fin[blockIdx.x];
  const int n = d.n, m = d.m;
  const int r0 = 16 * blockIdx.y;
  for (int r = r0; r < min(n, r0 + 16); ++r) {
    const int src = f.ord[r];
    if (d.U) {
      const double s = f.nrm[src];
      const double* a = d.A + (size_t)src * d.lda;
      double* u = d.U + (size_t)r * d.ldu;
      for (int i = threadIdx.x; i < m; i += 256) u[i] = s > 0 ? a[i] / s : 0.0;
    }
    if (d.V) {
      const double* v = d.V + (size_t)src * d.ldv;
      double* t = f.T + (size_t)r * n;
      for (int i = threadIdx.x; i < n; i += 256) t[i] = v[i];
    }
  }
}

__global__ __launch_bounds__(256) void k_svd_vback(const SVDDesc* __restrict__ descs,
                                                   const SvdFin* __restrict__ fin) {
  const SVDDesc d = descs[blockIdx.x];
  if (!d.V) return;
  const SvdFin f = fin[blockIdx.x];
  const int n = d.n;
  const int r0 = 16 * blockIdx.y;
  for (int r = r0; r < min(n, r0 + 16); ++r) {
    const double* t = f.T + (size_t)r * n;
    double* v = d.V + (size_t)r * d.ldv;
    for (int i = threadIdx.x; i < n; i += 256) v[i] = t[i];
  }
}

constexpr int SVD_COOP_MIN_N = 24;

// polls before a block Jacobi wait gives up (tests lower it to exercise the
// timeout path)
int svd_spin_limit = SVD_SPIN;

void svd_batched(Ctx& c, const std::vector<SVDDesc>& ds) {
  std::vector<SVDDesc> all, small, big;
  for (auto& d : ds) {
    if (d.n <= 0) continue;
    H2_CHECK(d.n <= 1024, H2_EINVAL, "SVD: more than 1024 columns");
    H2_CHECK(d.m >= d.n, H2_EINVAL, "SVD: needs m >= n");
    H2_CHECK(d.sigma != nullptr, H2_EINVAL, "SVD: sigma output required");
    all.push_back(d);
    (d.n >= SVD_COOP_MIN_N && d.m <= SVD_MMAX ? big : small).push_back(d);
  }
  if (all.empty()) return;
  auto* dall = (SVDDesc*)c.stage.put(all.data(), all.size() * sizeof(SVDDesc), c.s);
  int nmx = 1;
  for (auto& d : all) nmx = std::max(nmx, d.n);
  k_svd_init_v<<<dim3((unsigned)all.size(), (unsigned)((nmx + 15) / 16)), 256, 0, c.s>>>(dall);
  H2_LAUNCH_CHECK();
  if (!small.empty()) {
    auto* dd = (SVDDesc*)c.stage.put(small.data(), small.size() * sizeof(SVDDesc), c.s);
    k_svd_sweeps<<<(unsigned)small.size(), 512, 0, c.s>>>(dd);
    H2_LAUNCH_CHECK();
  }
  // status[0]: sweeps of the last launch, status[1]: synchronisation timeout
  int* status = (int*)c.scratch.get(1);
  H2_HIP(hipMemsetAsync(status, 0, 2 * sizeof(int), c.s));
  if (!big.empty()) {
    static int capacity = 0;
    if (capacity == 0) {
      int dev = 0, ncu = 0, per = 0;
      H2_HIP(hipGetDevice(&dev));
      H2_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      H2_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_svd_block, 512, 0));
      capacity = std::max(1, ncu * std::max(per, 1));
    }
    // launches of at most `capacity` co-resident workgroups, one block pair each
    size_t i0 = 0;
    while (i0 < big.size()) {
      size_t i1 = i0;
      int used = 0;
      std::vector<int> want;
      while (i1 < big.size()) {
        const int nb = (big[i1].n + SVD_BS - 1) / SVD_BS;
        const int w = (nb + (nb & 1)) / 2;
        if (used > 0 && used + w > capacity) break;
        want.push_back(std::min(w, capacity));
        used += want.back();
        ++i1;
      }
      const int nm = (int)(i1 - i0);
      std::vector<int> start(nm + 1, 0);
      int maxnb = 0;
      for (int j = 0; j < nm; ++j) {
        start[j + 1] = start[j] + want[j];
        maxnb = std::max(maxnb, (big[i0 + j].n + SVD_BS - 1) / SVD_BS);
      }
      auto* dd = (SVDDesc*)c.stage.put(big.data() + i0, nm * sizeof(SVDDesc), c.s);
      auto* dstart = (int*)c.stage.put(start.data(), start.size() * sizeof(int), c.s);
      // 3 nm rotation flags, nm * maxnb round counters, sweeps
      const size_t nint = (size_t)3 * nm + (size_t)nm * maxnb + 1;
      int* flags = (int*)c.scratch.get((nint + 1) / 2);
      H2_HIP(hipMemsetAsync(flags, 0, nint * sizeof(int), c.s));
      int* ver = flags + 3 * nm;
      int* sweeps = ver + (size_t)nm * maxnb;
      int nmi = nm;
      int spin = svd_spin_limit;
      void* args[] = {&dd, &dstart, &nmi, &maxnb, &flags, &ver, &status, &spin};
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (verbose()) {
        H2_HIP(hipEventCreate(&e0));
        H2_HIP(hipEventCreate(&e1));
        H2_HIP(hipEventRecord(e0, c.s));
      }
      // algorithmic work of a thin SVD with both factors (m x n, U1 m x n
      // and V n x n): 14 m n^2 + 8 n^3 flops (the Golub-Reinsch count of
      // Golub and Van Loan), independent of how many sweeps Jacobi takes
      double work = 0;
      for (int j = 0; j < nm; ++j) {
        const double n = big[i0 + j].n, m = big[i0 + j].m;
        work += 14.0 * m * n * n + 8.0 * n * n * n;
      }
      const int tok = timing_begin(c.s);
      H2_HIP(hipLaunchCooperativeKernel((const void*)k_svd_block, dim3(start[nm]), dim3(512), args,
                                        0, c.s));
      timing_end(tok, "k_svd_block", c.s, work, nullptr, 0.0);
      if (verbose()) {
        H2_HIP(hipEventRecord(e1, c.s));
        H2_HIP(hipEventSynchronize(e1));
        float ms = 0;
        H2_HIP(hipEventElapsedTime(&ms, e0, e1));
        int sw = 0;
        H2_HIP(hipMemcpy(&sw, status, sizeof(int), hipMemcpyDeviceToHost));
        std::fprintf(stderr, "    [svd] %d matrices, n %d..%d, m %d, %d workgroups: %d sweeps, %.2f ms\n",
                     nm, big[i0].n, big[i1 - 1].n, big[i0].m, start[nm], sw, ms);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
      }
      i0 = i1;
    }
  }
  std::vector<SvdFin> fin(all.size());
  int nmax = 1;
  for (size_t i = 0; i < all.size(); ++i) {
    const int n = all[i].n;
    nmax = std::max(nmax, n);
    fin[i].ord = (int*)c.scratch.get((size_t)(n + 1) / 2);
    fin[i].nrm = c.scratch.get((size_t)n);
    fin[i].T = all[i].V ? c.scratch.get((size_t)n * n) : nullptr;
  }
  auto* dfin = (SvdFin*)c.stage.put(fin.data(), fin.size() * sizeof(SvdFin), c.s);
  k_svd_order<<<(unsigned)all.size(), 1024, 0, c.s>>>(dall, dfin, status);
  const dim3 g2((unsigned)all.size(), (unsigned)((nmax + 15) / 16));
  k_svd_permute<<<g2, 256, 0, c.s>>>(dall, dfin);
  k_svd_vback<<<g2, 256, 0, c.s>>>(dall, dfin);
  H2_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ TSQR
// Tall-skinny Householder QR (n <= 96 columns): row chunks of at most 320
// rows are factorised by one workgroup each, groups of up to 320 / n of the R
// factors are stacked and factorised again up the tree, and the explicit Q is
// formed top-down by batched GEMMs (Q = diag(Q_chunks) * ... * Q_root).
// Backward stable for any rank, like a single Householder QR.  A node's time
// is set by its column count (one reflector per barrier), not by its rows, so
// nodes are as tall as the registers allow: fewer tree levels, fewer launches.
constexpr int TS_W = 96, TS_ROWS = 320, TS_SRC = 8;

struct TsqrNode {
  const double* src[TS_SRC];  // stacked row blocks, rs rows each
  int lds[TS_SRC];
  int nsrc, rs;
  int w;
  double* Q;          // (nsrc * rs) x w explicit Q (optional)
  int ldq;
  double* R;          // w x w, zero below the diagonal
  int ldr;
  const int* run;     // optional: the node does nothing when *run == 0
};

// One node = Householder QR of a stacked (nsrc * rs) x w block, rows <= 64 RS,
// w <= 96, held in registers: wave v owns columns v, v + 16, ... (at most 6),
// lane l holds rows l, l + 64, ..., l + 64 (RS - 1) (RS = 3 for nodes of at
// most 192 rows, else 5).  Per column j the owner wave forms the
// reflector and publishes it through LDS (double-buffered); after one barrier
// every wave applies it to its own columns, the owner of the next column
// first (see the factorisation loop).  The explicit Q (when requested) is
// accumulated backwards the same way: Q = H_0 ... H_{w-1} [I; 0].
constexpr int TS_WAVES = 16, TS_CPW = (TS_W + TS_WAVES - 1) / TS_WAVES, TS_RS_MAX = 5;
static_assert(TS_RS_MAX * 64 >= TS_ROWS, "node rows must fit the lanes");

// reflector of column j (rows held as col[r] = row r * 64 + lane): v below the
// diagonal (v_j = 1) stays in col, beta goes on the diagonal; v and tau are
// published to vb (rows) and tb (one value); returns tau
template <int TS_RS>
__device__ __forceinline__ double tsqr_reflect(double (&col)[TS_RS], int j, int lane, double* vb,
                                               double* tb) {
  double s = 0.0, alpha = 0.0;
#pragma unroll
  for (int r = 0; r < TS_RS; ++r) {
    const int i = r * 64 + lane;
    if (i > j) s += col[r] * col[r];
    if (i == j) alpha = col[r];
  }
  s = wave_sum(s);
  alpha = readlane_f64(alpha, j & 63);
  double tau = 0.0, scale = 0.0, beta = alpha;
  if (s != 0.0) {
    const double norm = sqrt(alpha * alpha + s);
    beta = alpha >= 0 ? -norm : norm;
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
#pragma unroll
  for (int r = 0; r < TS_RS; ++r) {
    const int i = r * 64 + lane;
    double v = 0.0;
    if (i > j) {
      if (s != 0.0) col[r] *= scale;
      v = col[r];
    } else if (i == j) {
      col[r] = beta;
      v = 1.0;
    }
    vb[i] = v;
  }
  if (lane == 0) *tb = tau;
  return tau;
}

// explicit-Q set-up of column j: publish v_j and tau, column := e_j - tau v_j
template <int TS_RS>
__device__ __forceinline__ void tsqr_publish(double (&col)[TS_RS], double tau, int j, int lane, double* vb,
                                             double* tb) {
#pragma unroll
  for (int r = 0; r < TS_RS; ++r) {
    const int i = r * 64 + lane;
    double v = 0.0;
    if (i > j) v = col[r];
    else if (i == j) v = 1.0;
    vb[i] = v;
    col[r] = (i == j ? 1.0 : 0.0) - tau * v;
  }
  if (lane == 0) *tb = tau;
}

template <int TS_RS, class NA>
__global__ __launch_bounds__(1024) void k_tsqr_node(NA nodes) {
  const TsqrNode& d = nodes[blockIdx.x];
  if (d.run && *d.run == 0) return;
  __shared__ double vbuf[2][TS_RS * 64];
  __shared__ double tbuf[2];
  __shared__ const double* rowp[TS_RS * 64];   // start of row i in its source
  __shared__ int rowld[TS_RS * 64];
  const int rs = d.rs, m = d.nsrc * rs, w = d.w;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < m) {
    const int sb = threadIdx.x / rs;
    rowp[threadIdx.x] = d.src[sb] + (threadIdx.x - sb * rs);
    rowld[threadIdx.x] = d.lds[sb];
  }
  __syncthreads();
  double a[TS_CPW][TS_RS];
  const double* rp[TS_RS];
  int rl[TS_RS];
#pragma unroll
  for (int r = 0; r < TS_RS; ++r) {
    const int i = r * 64 + lane;
    rp[r] = i < m ? rowp[i] : nullptr;
    rl[r] = i < m ? rowld[i] : 0;
  }
#pragma unroll
  for (int q = 0; q < TS_CPW; ++q) {
    const int c = wave + TS_WAVES * q;
#pragma unroll
    for (int r = 0; r < TS_RS; ++r) a[q][r] = (c < w && rp[r]) ? rp[r][(size_t)c * rl[r]] : 0.0;
  }
  double taus_own[TS_CPW];
#pragma unroll
  for (int q = 0; q < TS_CPW; ++q) taus_own[q] = 0.0;
  // ---- factorisation.  Step j applies H_j to the columns right of j; the
  // owner of column j + 1 updates that column first and forms reflector j + 1
  // at raised priority, so the next step's reflector is ready at the barrier.
  if (wave == 0 && w > 0) taus_own[0] = tsqr_reflect(a[0], 0, lane, vbuf[0], &tbuf[0]);
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    const int buf = j & 1;
    const double tau = tbuf[buf];
    double v[TS_RS];
#pragma unroll
    for (int r = 0; r < TS_RS; ++r) v[r] = vbuf[buf][r * 64 + lane];
    const int nx = j + 1, qn = nx / TS_WAVES;
    const bool lead = wave == nx % TS_WAVES && nx < w;
    if (lead) {
      __builtin_amdgcn_s_setprio(3);
#pragma unroll
      for (int q = 0; q < TS_CPW; ++q) {
        if (q != qn) continue;
        if (tau != 0.0) {
          double t = 0.0;
#pragma unroll
          for (int r = 0; r < TS_RS; ++r) t += v[r] * a[q][r];
          t = wave_sum(t) * tau;
#pragma unroll
          for (int r = 0; r < TS_RS; ++r) a[q][r] -= v[r] * t;
        }
        taus_own[q] = tsqr_reflect(a[q], nx, lane, vbuf[nx & 1], &tbuf[nx & 1]);
      }
      __builtin_amdgcn_s_setprio(0);
    }
    if (tau != 0.0) {
      double dot[TS_CPW];
#pragma unroll
      for (int q = 0; q < TS_CPW; ++q) {
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < TS_RS; ++r) t += v[r] * a[q][r];
        dot[q] = t;
      }
#pragma unroll
      for (int q = 0; q < TS_CPW; ++q) {
        const int c = wave + TS_WAVES * q;
        if (c > j && c < w && !(lead && q == qn)) {
          const double t = wave_sum(dot[q]) * tau;
#pragma unroll
          for (int r = 0; r < TS_RS; ++r) a[q][r] -= v[r] * t;
        }
      }
    }
    __syncthreads();
  }
  // R (w x w, upper triangular)
#pragma unroll
  for (int q = 0; q < TS_CPW; ++q) {
    const int c = wave + TS_WAVES * q;
    if (c >= w) continue;
    for (int i = lane; i < w; i += 64) {
      double x = 0.0;
#pragma unroll
      for (int r = 0; r < TS_RS; ++r)
        if (r * 64 + lane == i) x = a[q][r];
      d.R[(size_t)c * d.ldr + i] = i <= c ? x : 0.0;
    }
  }
  if (!d.Q) return;
  // ---- explicit Q = H_0 ... H_{w-1} [I; 0], backwards.  Column j of Q is
  // H_j e_j = e_j - tau_j v_j when step j begins; step j applies H_j to the
  // columns right of j.  The owner of column j - 1 publishes its reflector and
  // sets up that column during step j (it takes no part in step j).
  if (w > 0 && wave == (w - 1) % TS_WAVES) {
#pragma unroll
    for (int q = 0; q < TS_CPW; ++q)
      if (q == (w - 1) / TS_WAVES) tsqr_publish(a[q], taus_own[q], w - 1, lane, vbuf[(w - 1) & 1], &tbuf[(w - 1) & 1]);
  }
  __syncthreads();
  for (int j = w - 1; j >= 0; --j) {
    const int buf = j & 1;
    const double tau = tbuf[buf];
    double v[TS_RS];
#pragma unroll
    for (int r = 0; r < TS_RS; ++r) v[r] = vbuf[buf][r * 64 + lane];
    const int pv = j - 1;
    if (pv >= 0 && wave == pv % TS_WAVES) {
#pragma unroll
      for (int q = 0; q < TS_CPW; ++q)
        if (q == pv / TS_WAVES) tsqr_publish(a[q], taus_own[q], pv, lane, vbuf[pv & 1], &tbuf[pv & 1]);
    }
    if (tau != 0.0) {
      double dot[TS_CPW];
#pragma unroll
      for (int q = 0; q < TS_CPW; ++q) {
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < TS_RS; ++r) t += v[r] * a[q][r];
        dot[q] = t;
      }
#pragma unroll
      for (int q = 0; q < TS_CPW; ++q) {
        const int c = wave + TS_WAVES * q;
        if (c > j && c < w) {
          const double t = wave_sum(dot[q]) * tau;
#pragma unroll
          for (int r = 0; r < TS_RS; ++r) a[q][r] -= v[r] * t;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < TS_CPW; ++q) {
    const int c = wave + TS_WAVES * q;
    if (c >= w) continue;
#pragma unroll
    for (int r = 0; r < TS_RS; ++r) {
      const int i = r * 64 + lane;
      if (i < m) d.Q[(size_t)c * d.ldq + i] = a[q][r];
    }
  }
}

static void launch_nodes(Ctx& c, const std::vector<TsqrNode>& v) {
  if (v.empty()) return;
  for (auto& nd : v)
    H2_CHECK(nd.w <= TS_W && nd.nsrc >= 1 && nd.nsrc <= TS_SRC && nd.rs >= 1 &&
                 nd.nsrc * nd.rs <= TS_ROWS && nd.nsrc * nd.rs >= nd.w, H2_EINVAL,
             "TSQR node shape out of range");
  int rmax = 0;
  for (auto& nd : v) rmax = std::max(rmax, nd.nsrc * nd.rs);
  VTimer vt(c.s);
  with_descs<16>(c, v.data(), v.size(), [&](auto nodes) {
    if (rmax <= 192) k_tsqr_node<3><<<(unsigned)v.size(), 1024, 0, c.s>>>(nodes);
    else k_tsqr_node<TS_RS_MAX><<<(unsigned)v.size(), 1024, 0, c.s>>>(nodes);
  });
  H2_LAUNCH_CHECK();
  if (vt.on()) {
    int w = 0, rows = 0, q = 0;
    for (auto& nd : v) {
      w = std::max(w, nd.w);
      rows = std::max(rows, nd.nsrc * nd.rs);
      q += nd.Q != nullptr;
    }
    std::fprintf(stderr, "    [tsqr node] %zu nodes, w %d, rows %d, %d with Q: %.3f ms\n", v.size(), w, rows,
                 q, vt.stop());
  }
}

void qr_tall_batched(Ctx& c, const std::vector<QRDesc>& ds) {
  // per matrix: the tree of nodes (level 0 = chunks); a node of level l >= 1
  // stacks the R factors of up to `fan` consecutive nodes of level l - 1
  struct Mat {
    QRDesc d;
    int fan = 2;
    std::vector<int> chunk_rows;               // level 0
    std::vector<std::vector<double*>> Qs, Rs;
    std::vector<std::vector<int>> nchild;      // children per node (1: R passed through)
    bool r_direct = false;                     // the root wrote R into the output
  };
  std::vector<Mat> mats;
  for (auto& d : ds) {
    if (d.m <= 0 || d.n <= 0) continue;
    H2_CHECK(d.n <= TS_W && d.m >= d.n && (d.Q != nullptr || d.R != nullptr), H2_EINVAL,
             "TSQR: needs n <= 96, m >= n, Q or R");
    Mat M;
    M.d = d;
    M.fan = std::min(TS_SRC, TS_ROWS / d.n);
    // chunks of at most TS_ROWS rows and at least n rows, sizes balanced
    int nch = (d.m + TS_ROWS - 1) / TS_ROWS;
    while (nch > 1 && d.m / nch < d.n) --nch;
    for (int i = 0; i < nch; ++i) M.chunk_rows.push_back(d.m / nch + (i < d.m % nch ? 1 : 0));
    mats.push_back(std::move(M));
  }
  if (mats.empty()) return;
  // upward: level 0 chunks
  {
    std::vector<TsqrNode> nodes;
    for (auto& M : mats) {
      const int w = M.d.n;
      M.Qs.push_back({});
      M.Rs.push_back({});
      M.nchild.push_back(std::vector<int>(M.chunk_rows.size(), 0));
      // a matrix of one chunk is factorised by that node alone, which writes
      // the outputs directly (a node reads all of its rows before it writes)
      const bool single = M.chunk_rows.size() == 1;
      M.r_direct = single && M.d.R != nullptr;
      int r0 = 0;
      for (int rows : M.chunk_rows) {
        double* Q = M.d.Q ? (single ? M.d.Q : c.scratch.get((size_t)rows * w)) : nullptr;
        double* R = M.r_direct ? M.d.R : c.scratch.get((size_t)w * w);
        M.Qs[0].push_back(Q);
        M.Rs[0].push_back(R);
        TsqrNode nd{};
        nd.src[0] = M.d.A + r0;
        nd.lds[0] = M.d.lda;
        nd.nsrc = 1;
        nd.rs = rows;
        nd.w = w;
        nd.Q = Q;
        nd.ldq = single ? M.d.ldq : rows;
        nd.R = R;
        nd.ldr = M.r_direct ? M.d.ldr : w;
        nd.run = M.d.run;
        nodes.push_back(nd);
        r0 += rows;
      }
    }
    launch_nodes(c, nodes);
  }
  // upward: groups of R factors until one remains
  for (int lev = 1;; ++lev) {
    std::vector<TsqrNode> nodes;
    bool any = false;
    for (auto& M : mats) {
      const int w = M.d.n;
      // this matrix's tree may already be complete
      if ((int)M.Rs.size() < lev || M.Rs[lev - 1].size() == 1) continue;
      const std::vector<double*> prevR = M.Rs[lev - 1];   // copy: Rs grows below
      any = true;
      const int np = (int)prevR.size();
      const int cnt = (np + M.fan - 1) / M.fan;
      M.Qs.push_back({});
      M.Rs.push_back({});
      M.nchild.push_back(std::vector<int>(cnt, 0));
      for (int i = 0; i < cnt; ++i) {
        const int k0 = i * M.fan, k = std::min(M.fan, np - k0);
        M.nchild[lev][i] = k;
        if (k == 1) {
          M.Qs[lev].push_back(nullptr);
          M.Rs[lev].push_back(prevR[k0]);
          continue;
        }
        // the root (one node at this level) writes R into the output
        const bool root = cnt == 1 && M.d.R != nullptr;
        double* Q = M.d.Q ? c.scratch.get((size_t)k * w * w) : nullptr;
        double* R = root ? M.d.R : c.scratch.get((size_t)w * w);
        M.r_direct = M.r_direct || root;
        M.Qs[lev].push_back(Q);
        M.Rs[lev].push_back(R);
        TsqrNode nd{};
        for (int j = 0; j < k; ++j) {
          nd.src[j] = prevR[k0 + j];
          nd.lds[j] = w;
        }
        nd.nsrc = k;
        nd.rs = w;
        nd.w = w;
        nd.Q = Q;
        nd.ldq = k * w;
        nd.R = R;
        nd.ldr = root ? M.d.ldr : w;
        nd.run = M.d.run;
        nodes.push_back(nd);
      }
    }
    if (!any) break;
    launch_nodes(c, nodes);
  }
  // (R: written by the root, or by the chunk's node for a matrix of one chunk)
  // downward: X (w x w) per node; the root's children take their rows of the
  // root's Q (X = I at the root).  Matrices of one chunk are complete.
  mats.erase(std::remove_if(mats.begin(), mats.end(),
                            [](const Mat& M) { return M.d.Q == nullptr || M.chunk_rows.size() == 1; }),
             mats.end());
  if (mats.empty()) return;
  int maxlev = 0;
  for (auto& M : mats) maxlev = std::max(maxlev, (int)M.Rs.size() - 1);
  std::vector<std::vector<std::vector<const double*>>> X(mats.size());
  std::vector<std::vector<std::vector<int>>> ldx(mats.size());
  for (size_t mi = 0; mi < mats.size(); ++mi) {
    const int top = (int)mats[mi].Rs.size() - 1;
    X[mi].assign(top + 1, {});
    ldx[mi].assign(top + 1, {});
  }
  for (int lev = maxlev; lev >= 1; --lev) {
    std::vector<GemmDesc> g;
    for (size_t mi = 0; mi < mats.size(); ++mi) {
      auto& M = mats[mi];
      const int top = (int)M.Rs.size() - 1, w = M.d.n;
      if (lev > top) continue;
      const size_t cnt = M.Rs[lev].size();
      X[mi][lev - 1].assign(M.Rs[lev - 1].size(), nullptr);
      ldx[mi][lev - 1].assign(M.Rs[lev - 1].size(), w);
      for (size_t i = 0; i < cnt; ++i) {
        const int k = M.nchild[lev][i], k0 = (int)i * M.fan;
        if (k == 1) {  // R passed through: the child keeps this X
          X[mi][lev - 1][k0] = X[mi][lev][i];
          ldx[mi][lev - 1][k0] = ldx[mi][lev][i];
          continue;
        }
        if (lev == top) {  // the root: Q_root I = Q_root
          for (int j = 0; j < k; ++j) {
            X[mi][lev - 1][k0 + j] = M.Qs[lev][i] + (size_t)j * w;
            ldx[mi][lev - 1][k0 + j] = k * w;
          }
          continue;
        }
        double* Y = c.scratch.get((size_t)k * w * w);
        g.push_back({M.Qs[lev][i], X[mi][lev][i], Y, k * w, w, w, k * w, ldx[mi][lev][i], k * w, 0, 0, 1.0, 0.0,
                     M.d.run});
        for (int j = 0; j < k; ++j) {
          X[mi][lev - 1][k0 + j] = Y + (size_t)j * w;
          ldx[mi][lev - 1][k0 + j] = k * w;
        }
      }
    }
    gemm_batched(c, g);
  }
  // level 0: Q rows of each chunk = Q_chunk X
  std::vector<GemmDesc> g;
  for (size_t mi = 0; mi < mats.size(); ++mi) {
    auto& M = mats[mi];
    const int w = M.d.n;
    int r0 = 0;
    for (size_t i = 0; i < M.chunk_rows.size(); ++i) {
      const int rows = M.chunk_rows[i];
      g.push_back({M.Qs[0][i], X[mi][0][i], M.d.Q + r0, rows, w, w, rows, ldx[mi][0][i], M.d.ldq, 0, 0, 1.0, 0.0,
                   M.d.run});
      r0 += rows;
    }
  }
  gemm_batched(c, g);
}

void qr_blocked(Ctx& c, const std::vector<CholQRDesc>& ds) {
  // block Gram-Schmidt with reorthogonalisation of the normalised block
  // (BCGS2):  S1 = Q^T P, P -= Q S1, P = Q1 R1;  S2 = Q^T Q1, Q1 -= Q S2,
  // Q1 = Q2 R2;  R_jj = R2 R1,  R[0:j0, j] = S1 + S2 R1.  Stable when the
  // panel is numerically dependent on the previous ones, except for the
  // columns of Q1 that lie in the span of Q (a rank-deficient panel's QR
  // completes its basis with such columns, whose rows of R1 are at rounding
  // level): those are replaced by Gaussian directions and projected once more
  // (S3 = Q^T Q1, Q1 -= Q S3, S2 += S3) before Q1 = Q2 R2.
  constexpr int W = 64;
  int maxp = 0;
  std::vector<CholQRDesc> v;
  for (auto& d : ds)
    if (d.m > 0 && d.n > 0) {
      H2_CHECK(d.m >= d.n && d.R != nullptr, H2_EINVAL, "blocked QR needs m >= n and R");
      v.push_back(d);
      maxp = std::max(maxp, (d.n + W - 1) / W);
    }
  if (v.empty()) return;
  {
    // R = 0 for every matrix in one launch (empty products write zeros)
    std::vector<GemmDesc> zr;
    for (auto& d : v) zr.push_back({nullptr, nullptr, d.R, d.n, d.n, 0, 1, 1, d.ldr, 0, 0, 1.0, 0.0});
    gemm_batched(c, zr);
  }
  for (int j = 0; j < maxp; ++j) {
    // a panel's temporaries (and those of its tall QRs) are dead once its
    // results are in P and R: the next panel reuses their memory
    const Scratch::Mark panel_mark = c.scratch.mark();
    std::vector<GemmDesc> p1, p2, p3, p4, p6, p7, rr, rs, rs3;
    std::vector<QRDesc> tq1, tq2;
    std::vector<CopyDesc> back, lost;
    std::vector<uint64_t> lost_keys;
    for (auto& d : v) {
      const int j0 = j * W;
      if (j0 >= d.n) continue;
      const int w = std::min(W, d.n - j0);
      double* Pj = d.P + (size_t)j0 * d.ld;
      double* Rj = d.R + (size_t)j0 * d.ldr;      // R[0:j0, j0:j0+w]
      double* Rjj = Rj + j0;
      double* Q1 = c.scratch.get((size_t)d.m * w);
      if (j0 == 0) {
        tq1.push_back({Pj, d.ld, d.m, w, Q1, d.m, Rjj, d.ldr});
        back.push_back({Q1, d.m, Pj, d.ld, d.m, w, 1.0, 0.0, 0});
        continue;
      }
      double* R1 = c.scratch.get((size_t)w * w);
      double* R2 = c.scratch.get((size_t)w * w);
      double* S2 = c.scratch.get((size_t)j0 * w);
      double* S3 = c.scratch.get((size_t)j0 * w);
      double* Q2 = c.scratch.get((size_t)d.m * w);
      p1.push_back({d.P, Pj, Rj, j0, w, d.m, d.ld, d.ld, d.ldr, 1, 0, 1.0, 0.0});      // S1
      p2.push_back({d.P, Rj, Pj, d.m, w, j0, d.ld, d.ldr, d.ld, 0, 0, -1.0, 1.0});     // P -= Q S1
      tq1.push_back({Pj, d.ld, d.m, w, Q1, d.m, R1, w});                                // P = Q1 R1
      p3.push_back({d.P, Q1, S2, j0, w, d.m, d.ld, d.m, j0, 1, 0, 1.0, 0.0});          // S2
      p4.push_back({d.P, S2, Q1, d.m, w, j0, d.ld, j0, d.m, 0, 0, -1.0, 1.0});         // Q1 -= Q S2
      // columns of Q1 that the projection removed (dependent panel) become
      // Gaussian; one more projection, whose coefficients S3 enter R like S2
      // (these three products run only for blocks with a replaced column)
      lost.push_back({Q1, d.m, nullptr, 0, d.m, w, 1.0, 0.0, 0});
      lost_keys.push_back(stream_key(0x9e3779b97f4a7c15ull ^ (uint64_t)d.m, PHASE_LOST, (uint32_t)j,
                                     (uint32_t)d.n, (uint32_t)v.size()));
      p6.push_back({d.P, Q1, S3, j0, w, d.m, d.ld, d.m, j0, 1, 0, 1.0, 0.0});          // S3 = Q^T Q1
      p7.push_back({d.P, S3, Q1, d.m, w, j0, d.ld, j0, d.m, 0, 0, -1.0, 1.0});         // Q1 -= Q S3
      tq2.push_back({Q1, d.m, d.m, w, Q2, d.m, R2, w});                                 // Q1 = Q2 R2
      rr.push_back({R2, R1, Rjj, w, w, w, w, w, d.ldr, 0, 0, 1.0, 0.0});                // R_jj
      rs.push_back({S2, R1, Rj, j0, w, w, j0, w, d.ldr, 0, 0, 1.0, 1.0});               // S1 += S2 R1
      rs3.push_back({S3, R1, Rj, j0, w, w, j0, w, d.ldr, 0, 0, 1.0, 1.0});              // ... + S3 R1
      back.push_back({Q2, d.m, Pj, d.ld, d.m, w, 1.0, 0.0, 0});
    }
    // lost-column flags: p6, p7 and the S3 R1 term run only where a column was replaced
    int* flags = nullptr;
    if (!lost.empty()) {
      flags = (int*)c.scratch.get((lost.size() + 1) / 2);
      zero_block(c, (double*)flags, (int)((lost.size() + 1) / 2), 1, (int)((lost.size() + 1) / 2));
      for (size_t i = 0; i < lost.size(); ++i) {
        p6[i].run = flags + i;
        p7[i].run = flags + i;
        rs3[i].run = flags + i;
      }
    }
    gemm_batched(c, p1);
    gemm_batched(c, p2);
    qr_tall_batched(c, tq1);
    gemm_batched(c, p3);
    gemm_batched(c, p4);
    replace_lost_columns(c, lost, lost_keys, flags);
    gemm_batched(c, p6);
    gemm_batched(c, p7);
    qr_tall_batched(c, tq2);
    gemm_batched(c, rr);
    gemm_batched(c, rs);
    gemm_batched(c, rs3);
    copy_batched(c, back);
    c.scratch.release(panel_mark);
  }
}

void qr_auto(Ctx& c, const std::vector<QRDesc>& ds) {
  std::vector<QRDesc> small, tall;
  std::vector<CholQRDesc> blocked;
  std::vector<CopyDesc> toq;
  std::vector<GemmDesc> wide_r, wide_r2;   // R(:, m:) = Q^T A(:, m:) of wide matrices
  std::vector<CopyDesc> toq2;
  for (auto d : ds) {
    if (d.m <= 0 || d.n <= 0) continue;
    H2_CHECK(d.run == nullptr, H2_EINVAL, "QR run flags are taken by the tall QR only");
    if (d.m < d.n) {
      // wide: the m reflectors come from the first m columns, so Q is the Q of
      // those columns (TSQR) and R = [R_1, Q^T A(:, m:)] (one GEMM)
      if (d.m <= TS_W) {
        QRDesc e = d;
        e.n = d.m;
        if (d.R != nullptr) {
          double* Q = d.Q ? d.Q : c.scratch.get((size_t)d.m * d.m);
          const int ldq = d.Q ? d.ldq : d.m;
          e.Q = Q;
          e.ldq = ldq;
          wide_r.push_back({Q, d.A + (size_t)d.m * d.lda, d.R + (size_t)d.m * d.ldr, d.m, d.n - d.m, d.m,
                            ldq, d.lda, d.ldr, 1, 0, 1.0, 0.0});
        }
        tall.push_back(e);
      } else {
        // blocked QR of the first m columns in place (A(:, :m) becomes Q)
        double* R = d.R ? d.R : c.scratch.get((size_t)d.m * d.m);
        const int ldr = d.R ? d.ldr : d.m;
        blocked.push_back({d.A, d.lda, d.m, d.m, R, ldr});
        if (d.R)
          wide_r2.push_back({d.A, d.A + (size_t)d.m * d.lda, d.R + (size_t)d.m * d.ldr, d.m, d.n - d.m, d.m,
                             d.lda, d.lda, d.ldr, 1, 0, 1.0, 0.0});
        if (d.Q) toq2.push_back({d.A, d.lda, d.Q, d.ldq, d.m, d.m, 1.0, 0.0, 0});
      }
    } else if (d.n <= TS_W) {
      tall.push_back(d);
    } else {
      double* P = d.A;
      int ld = d.lda;
      if (d.Q && d.Q != d.A) {
        toq.push_back({d.A, d.lda, d.Q, d.ldq, d.m, d.n, 1.0, 0.0, 0});
        P = d.Q;
        ld = d.ldq;
      }
      double* R = d.R;
      int ldr = d.ldr;
      if (!R) {
        R = c.scratch.get((size_t)d.n * d.n);
        ldr = d.n;
      }
      blocked.push_back({P, ld, d.m, d.n, R, ldr});
    }
  }
  VTimer vt(c.s);
  qr_batched(c, small);
  qr_tall_batched(c, tall);
  gemm_batched(c, wide_r);
  copy_batched(c, toq);
  qr_blocked(c, blocked);
  gemm_batched(c, wide_r2);
  copy_batched(c, toq2);
  if (vt.on() && !(small.empty() && tall.empty() && blocked.empty())) {
    int mm = 0, mn = 0;
    for (auto& d : ds) { mm = std::max(mm, d.m); mn = std::max(mn, d.n); }
    std::fprintf(stderr, "    [qr] %zu one-wg, %zu tsqr, %zu blocked; max %d x %d: %.2f ms\n",
                 small.size(), tall.size(), blocked.size(), mm, mn, vt.stop());
  }
}

// ------------------------------------------------------------------ copies, norms
template <class CA>
__global__ void k_copy(CA ds) {
  const CopyDesc d = ds[blockIdx.y];
  const int64_t tot = (int64_t)d.rows * d.cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % d.rows), j = (int)(e / d.rows);
    const double v = d.trans ? d.src[(size_t)i * d.lds + j] : d.src[(size_t)j * d.lds + i];
    double* o = d.dst + (size_t)j * d.ldd + i;
    *o = d.beta == 0.0 ? d.alpha * v : d.alpha * v + d.beta * *o;
  }
}

void copy_batched(Ctx& c, const std::vector<CopyDesc>& ds) {
  std::vector<CopyDesc> v;
  int64_t mx = 0;
  for (auto& d : ds)
    if (d.rows > 0 && d.cols > 0) {
      v.push_back(d);
      mx = std::max(mx, (int64_t)d.rows * d.cols);
    }
  if (v.empty()) return;
  // one grid row per descriptor: launches of at most 65535 descriptors
  for (size_t i0 = 0; i0 < v.size(); i0 += 65535) {
    const size_t cnt = std::min<size_t>(65535, v.size() - i0);
    dim3 grid((unsigned)std::min<int64_t>((mx + 255) / 256, 1024), (unsigned)cnt);
    with_descs<40>(c, v.data() + i0, cnt, [&](auto dd) { k_copy<<<grid, 256, 0, c.s>>>(dd); });
    H2_LAUNCH_CHECK();
  }
}

template <class CA>
__global__ __launch_bounds__(1024) void k_colnorm_max(CA ds, double* __restrict__ out) {
  // one wave per column, 16 waves
  const CopyDesc d = ds[blockIdx.x];
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double best = 0;
  for (int j = wave; j < d.cols; j += 16) {
    const double* col = d.src + (size_t)j * d.lds;
    double s = 0;
    for (int i = lane; i < d.rows; i += 64) s += col[i] * col[i];
    s = wave_sum(s);
    best = fmax(best, sqrt(s));
  }
  if (lane == 0) red[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < 16; ++w) m = fmax(m, red[w]);
    out[blockIdx.x] = m;
  }
}

// Columns of a projected orthonormal block that lie (numerically) in the
// span that was projected out carry no direction of their own: for a
// rank-deficient block, Householder QR completes the basis with unit vectors
// of the block's own coordinates, which may lie in that span.  A column is
// lost when its norm fell below 1/2 (dst == nullptr: the block itself is
// tested), or, for the Q factor of a QR of the projected block, when the
// diagonal entry of its R (dst, ldd) is below 1/2 in magnitude (dependent on
// the span or on the block's earlier columns).  A lost column is replaced by
// a Gaussian vector of about unit norm (keyed by the block's key, row and
// column), so that the projection and QR that follow give a direction
// orthogonal to the span.  One wave per column.
template <class CA, class KA>
__global__ __launch_bounds__(256) void k_replace_lost_columns(CA ds, KA keys, int* __restrict__ flags,
                                                              int* __restrict__ nlost) {
  const CopyDesc d = ds[blockIdx.x];
  const uint64_t key = keys[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* X = const_cast<double*>(d.src);
  const double sc = 1.0 / sqrt((double)max(d.rows, 1));
  for (int j = wave + 4 * blockIdx.y; j < d.cols; j += 4 * gridDim.y) {
    double* col = X + (size_t)j * d.lds;
    bool lost;
    if (d.dst) {
      lost = fabs(d.dst[(size_t)j * d.ldd + j]) < 0.5;
    } else {
      double s = 0;
      for (int i = lane; i < d.rows; i += 64) s += col[i] * col[i];
      lost = wave_sum(s) < 0.25;
    }
    if (lost) {
      for (int i = lane; i < d.rows; i += 64) col[i] = sc * gauss_entry(key, (uint64_t)i, (uint64_t)j);
      if (flags && lane == 0) flags[blockIdx.x] = 1;
      if (nlost && lane == 0) atomicAdd(nlost, 1);
    }
  }
}

void replace_lost_columns(Ctx& c, const std::vector<CopyDesc>& blocks,
                          const std::vector<uint64_t>& keys, int* flags) {
  if (blocks.empty()) return;
  H2_CHECK(blocks.size() == keys.size(), H2_EINVAL, "one key per block");
  int mc = 1;
  for (auto& b : blocks) mc = std::max(mc, b.cols);
  const dim3 grid((unsigned)blocks.size(), (unsigned)((mc + 3) / 4));
  // verbose runs count the replaced columns
  int* nlost = nullptr;
  if (verbose()) {
    nlost = (int*)c.scratch.get(1);
    H2_HIP(hipMemsetAsync(nlost, 0, sizeof(int), c.s));
  }
  with_descs<32>(c, blocks.data(), blocks.size(), [&](auto dd) {
    with_descs<32>(c, keys.data(), keys.size(), [&](auto dk) {
      k_replace_lost_columns<<<grid, 256, 0, c.s>>>(dd, dk, flags, nlost);
    });
  });
  H2_LAUNCH_CHECK();
  if (nlost) {
    int n = 0, tot = 0;
    H2_HIP(hipMemcpyAsync(&n, nlost, sizeof(int), hipMemcpyDeviceToHost, c.s));
    H2_HIP(hipStreamSynchronize(c.s));
    for (auto& b : blocks) tot += b.cols;
    std::fprintf(stderr, "    [lost] %d of %d columns in %zu blocks\n", n, tot, blocks.size());
  }
}

void colnorm_max_batched(Ctx& c, const std::vector<CopyDesc>& blocks, double* out) {
  if (blocks.empty()) return;
  with_descs<40>(c, blocks.data(), blocks.size(), [&](auto dd) {
    k_colnorm_max<<<(unsigned)blocks.size(), 1024, 0, c.s>>>(dd, out);
  });
  H2_LAUNCH_CHECK();
}

__global__ void k_scale_cols(const ScaleDesc* __restrict__ ds) {
  const ScaleDesc d = ds[blockIdx.y];
  const int64_t tot = (int64_t)d.rows * d.cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % d.rows), j = (int)(e / d.rows);
    d.X[(size_t)j * d.ld + i] *= d.sigma[j];
  }
}

void scale_columns(Ctx& c, const std::vector<ScaleDesc>& ds) {
  if (ds.empty()) return;
  int64_t mx = 0;
  for (auto& d : ds) mx = std::max(mx, (int64_t)d.rows * d.cols);
  for (size_t i0 = 0; i0 < ds.size(); i0 += 65535) {
    const size_t cnt = std::min<size_t>(65535, ds.size() - i0);
    auto* dd = (ScaleDesc*)c.stage.put(ds.data() + i0, cnt * sizeof(ScaleDesc), c.s);
    dim3 grid((unsigned)std::min<int64_t>((mx + 255) / 256, 1024), (unsigned)cnt);
    k_scale_cols<<<grid, 256, 0, c.s>>>(dd);
    H2_LAUNCH_CHECK();
  }
}

// one block per matrix, one wave per column: arg-max of |x| (first index on
// ties), then the column is negated when that entry is negative
// one wave per column: blockIdx.y selects the block, blockIdx.x a group of 4 columns
__global__ __launch_bounds__(256) void k_canon_sign(const CopyDesc* __restrict__ ds) {
  const CopyDesc d = ds[blockIdx.y];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = 4 * blockIdx.x + wave;
  if (j >= d.cols) return;
  double* col = const_cast<double*>(d.src) + (size_t)j * d.lds;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int i = lane; i < d.rows; i += 64) {
    const double a = fabs(col[i]);
    if (a > best) { best = a; bi = i; }   // ascending i: keeps the first maximum
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  const bool flip = bi < d.rows && col[bi] < 0.0;
  if (flip)
    for (int i = lane; i < d.rows; i += 64) col[i] = -col[i];
}

void canonical_signs(Ctx& c, const std::vector<CopyDesc>& blocks) {
  std::vector<CopyDesc> v;
  for (auto& b : blocks)
    if (b.rows > 0 && b.cols > 0) v.push_back(b);
  if (v.empty()) return;
  int maxc = 0;
  for (auto& b : v) maxc = std::max(maxc, b.cols);
  for (size_t i0 = 0; i0 < v.size(); i0 += 65535) {
    const size_t cnt = std::min<size_t>(65535, v.size() - i0);
    auto* dd = (CopyDesc*)c.stage.put(v.data() + i0, cnt * sizeof(CopyDesc), c.s);
    k_canon_sign<<<dim3((unsigned)((maxc + 3) / 4), (unsigned)cnt), 256, 0, c.s>>>(dd);
    H2_LAUNCH_CHECK();
  }
}

__global__ void k_zero(double* p, int rows, int cols, int ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  p[(size_t)(e / rows) * ld + e % rows] = 0.0;
}

void zero_block(Ctx& c, double* p, int rows, int cols, int ld) {
  const int64_t tot = (int64_t)rows * cols;
  if (tot <= 0) return;
  k_zero<<<(unsigned)((tot + 255) / 256), 256, 0, c.s>>>(p, rows, cols, ld);
  H2_LAUNCH_CHECK();
}

}  // namespace h2
