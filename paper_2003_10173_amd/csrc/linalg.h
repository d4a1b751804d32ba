// Batched FP64 dense kernels of the construction (Sec. 3.3 sampling and
// compression phases): generic batched GEMM, Householder QR with explicit
// thin Q, one-sided Jacobi SVD, batched block copies and column norms.
#pragma once

#include <vector>

#include "internal.h"

namespace h2 {

// Pinned host + device ring used to ship descriptor arrays to kernels without
// synchronising the stream; a full ring is replaced by a fresh one and freed
// at the next reset().
struct Staging {
  char* host = nullptr;
  DevBuf dev;
  size_t cap = 0, head = 0;
  std::vector<char*> retired_host;   // full rings kept until reset()
  std::vector<DevBuf> retired_dev;
  explicit Staging(size_t cap_bytes = (size_t)32 << 20);
  ~Staging();
  Staging(const Staging&) = delete;
  Staging& operator=(const Staging&) = delete;
  void* put(const void* src, size_t bytes, hipStream_t s);
  void reset();  // only when the stream is known to be idle
};

// Grow-only scratch arena reused across launches of one driver call.
struct Scratch {
  std::vector<DevBuf> bufs;
  size_t used = 0;
  double* get(size_t elems);  // returns a fresh region valid until clear()
  void clear();               // only when the stream is idle
  // Stream-ordered reuse: release(mark()) hands the regions obtained after
  // the mark out again.  Every user of the arena enqueues on the one stream
  // of its context, so work enqueued later runs after the work that used
  // the released regions; the host must not read them afterwards.
  struct Mark { size_t nbufs, used; };
  Mark mark() const { return {bufs.size(), used}; }
  void release(const Mark& m) { used = bufs.size() == m.nbufs ? m.used : 0; }
};

// C (M x N) = alpha op(A) op(B) + beta C, column-major; op(X) = X or X^T.
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int lda, ldb, ldc;
  int ta, tb;
  double alpha, beta;
  const int* run = nullptr;  // optional device flag: the product is skipped when *run == 0
};

// In-place Householder QR of A (m x n): R (min(m,n) x n, upper) to R, explicit
// thin Q (m x min(m,n)) to Q when Q is non-null.  A keeps the reflectors.
struct QRDesc {
  double* A;
  int lda, m, n;
  double* Q;
  int ldq;
  double* R;
  int ldr;
  const int* run = nullptr;  // optional device flag, TSQR only: skipped when *run == 0
};

// One-sided Jacobi SVD of A (m x n, m >= n, destroyed): sigma descending (n),
// U (m x n) left singular vectors, V (n x n) right singular vectors (either may
// be null).
struct SVDDesc {
  double* A;
  int lda, m, n;
  double* sigma;
  double* U;
  int ldu;
  double* V;
  int ldv;
  // Jacobi tolerance: columns count as orthogonal once |a.b| <= tol |a| |b|;
  // 0 (or anything below it): the rounding level of an m-term FP64 dot
  // product.  Input known only to a lower precision (FP32 samples) needs no
  // sweeps that orthogonalise below that precision.
  double tol = 0.0;
};

// dst (rows x cols) = alpha * src (+ beta * dst), column-major blocks
struct CopyDesc {
  const double* src;
  int lds;
  double* dst;
  int ldd;
  int rows, cols;
  double alpha, beta;
  int trans;  // 1: dst = alpha src^T (src is cols x rows)
};

// In-place QR request: P (m x n, ld) is replaced by Q; R (n x n, upper) to R.
struct CholQRDesc {
  double* P;
  int ld, m, n;
  double* R;
  int ldr;
};

struct Ctx {
  hipStream_t s = 0;
  Staging stage;
  Scratch scratch;
  Ctx() = default;
};

// X[:, j] *= sigma[j] for a rows x cols block (column-major, ld)
struct ScaleDesc {
  double* X;
  int ld, rows, cols;
  const double* sigma;
};

void gemm_batched(Ctx& c, const std::vector<GemmDesc>& d);
// flip each column of X (rows x cols, ld) so that its largest-magnitude entry
// is positive (first index on ties); uses CopyDesc src/lds/rows/cols
void canonical_signs(Ctx& c, const std::vector<CopyDesc>& blocks);
void scale_columns(Ctx& c, const std::vector<ScaleDesc>& d);
void qr_batched(Ctx& c, const std::vector<QRDesc>& d);
void svd_batched(Ctx& c, const std::vector<SVDDesc>& d);
// polls before a wait of the multi-workgroup Jacobi gives up (singular values
// of that call come out as NaN); the default is a few seconds
extern int svd_spin_limit;
void copy_batched(Ctx& c, const std::vector<CopyDesc>& d);
// tall-skinny Householder QR by a TSQR tree (n <= 96, m >= n): explicit Q and R
void qr_tall_batched(Ctx& c, const std::vector<QRDesc>& d);
// blocked QR of tall matrices (m >= n): 64-column panels, two block
// Gram-Schmidt projections per panel by GEMM, TSQR per panel; P is
// replaced by Q (m x n) and R (n x n, upper) is written to R
void qr_blocked(Ctx& c, const std::vector<CholQRDesc>& d);
// QR of each matrix by the fastest applicable kernel: TSQR for m >= n and
// n <= 96, blocked QR for m >= n and n > 96; a wide matrix (m < n) is
// factorised through its first m columns (TSQR for m <= 96, blocked QR
// otherwise) with R(:, m:) = Q^T A(:, m:) by GEMM.  A is
// overwritten; Q (thin, optional) and R (optional, min(m,n) x n upper) as in
// QRDesc.
void qr_auto(Ctx& c, const std::vector<QRDesc>& d);
// columns of the blocks (CopyDesc src/lds/rows/cols, written in place) that
// lie in a span projected out become Gaussian vectors of about unit norm,
// keyed by keys[i], row and column: with dst == nullptr the columns of norm
// below 1/2; with dst/ldd the R of a QR whose Q the block is, the columns
// whose |R_jj| is below 1/2.  With flags (device, one int per block, zeroed
// by the caller), flags[i] becomes 1 when block i had a lost column.
void replace_lost_columns(Ctx& c, const std::vector<CopyDesc>& blocks,
                          const std::vector<uint64_t>& keys, int* flags = nullptr);
// out[i] = max_j || X_i[:, j] || for blocks X_i (rows_i x cols_i, ld_i)
void colnorm_max_batched(Ctx& c, const std::vector<CopyDesc>& blocks, double* out);
// zero a column-major block
void zero_block(Ctx& c, double* p, int rows, int cols, int ld);

}  // namespace h2
