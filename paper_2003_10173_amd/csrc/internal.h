// Internal declarations of the MI355X H2 library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "h2.h"

namespace h2 {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  h2_status status;
  Error(h2_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void set_last_error(const std::string& msg);
// progress trace to stderr when the environment sets H2_VERBOSE=1
bool verbose();

#define H2_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::h2::Error(H2_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_) +  \
                                        " at " + __FILE__ + ":" + std::to_string(__LINE__)); \
  } while (0)

#define H2_CHECK(cond, status, msg)                         \
  do {                                                      \
    if (!(cond)) throw ::h2::Error((status), (msg));        \
  } while (0)

#define H2_LAUNCH_CHECK() H2_HIP(hipGetLastError())

// ------------------------------------------------------------------ device memory
// RAII device buffer (hipMalloc / hipFree); size in bytes.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(H2_ENOMEM, "hipMalloc(" + std::to_string(b) + ") failed: " + hipGetErrorString(e));
    }
    bytes = b;
  }
  // grow-only reallocation (contents not preserved)
  void reserve(size_t b) { if (b > bytes) alloc(b); }
  void release() { if (p) { (void)hipFree(p); p = nullptr; bytes = 0; } }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

template <class T>
inline void upload(DevBuf& d, const std::vector<T>& h) {
  d.alloc(h.size() * sizeof(T));
  if (!h.empty()) H2_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

// ------------------------------------------------------------------ tree
// global cluster index of cluster i at level l
inline int cid(int l, int i) { return (1 << l) - 1 + i; }

}  // namespace h2

struct h2_tree {
  int n = 0, dim = 0, leaf = 0, L = 0;
  double eta = 0;
  std::vector<double> points;                       // n x dim, user order
  std::vector<int64_t> perm;                        // tree position -> user index
  std::vector<std::vector<int64_t>> offsets;        // per level, 2^l + 1
  std::vector<std::vector<double>> lo, hi;          // per level, 2^l x dim
  std::vector<std::vector<std::pair<int, int>>> far;  // per level, sorted (t, s)
  std::vector<std::pair<int, int>> near;            // leaf level, sorted
  // flattened per global cluster
  std::vector<int32_t> cstart, csize;               // per global cluster
  // far CSR per level (row cluster t): ptr has 2^l + 1 entries per level,
  // concatenated; far_base[l] = index of the level's first pair
  std::vector<int32_t> far_ptr, far_col;
  std::vector<int64_t> far_ptr_base, far_base;
  std::vector<int32_t> near_ptr, near_col;
  int max_leaf = 0;
  bool device_ready = false;
  // autotuned matrix-core tile width (16-column tiles per workgroup) of the
  // HGEMV stages of matrices on this tree, per (min(ceil(nv / 16), 4),
  // matrix element size, vector element size)
  mutable std::map<std::tuple<int, int, int>, int> tuned_nt;
  // device copies (made on first device use)
  h2::DevBuf d_perm, d_cstart, d_csize, d_far_ptr, d_far_col, d_near_ptr, d_near_col;
  int64_t num_far() const { return far_base.empty() ? 0 : far_base.back(); }
  int nclusters() const { return (2 << L) - 1; }
};

namespace h2 {

void tree_build(h2_tree* t);          // host: partition + lists
void tree_device(const h2_tree* t);   // device copies of the index arrays (idempotent)

// ------------------------------------------------------------------ matrices
// Element storage for H2 blocks; FP64 / FP32 / BF16 (raw uint16 bits).
struct Storage {
  h2_precision prec = H2_FP64;
  DevBuf U, E, S, D;
  size_t elem() const { return prec == H2_FP64 ? 8 : (prec == H2_FP32 ? 4 : 2); }
};

}  // namespace h2

struct h2_matrix {
  const h2_tree* tree = nullptr;
  std::vector<int32_t> rank;                        // per global cluster
  std::vector<int64_t> U_off, E_off, S_off, D_off;  // element offsets (+ total at end)
  std::vector<int64_t> kpre;                        // prefix of ranks per cluster (+ total)
  int kmax = 0;
  h2::Storage st;
  h2::DevBuf d_rank, d_U_off, d_E_off, d_S_off, d_D_off, d_kpre;
  // HGEMV workspace (grown on demand): tree-order x, y and coefficient vectors
  mutable h2::DevBuf ws;
  mutable h2::DevBuf ws_vec;  // user <-> tree order staging of h2_gemv
  // arrival counters of the split block rows (zero between products)
  mutable h2::DevBuf ws_cnt;
  int64_t nU() const { return U_off.back(); }
  int64_t nE() const { return E_off.back(); }
  int64_t nS() const { return S_off.back(); }
  int64_t nD() const { return D_off.back(); }
};

namespace h2 {

// layout helpers (host): fill offsets from ranks, upload index arrays
void matrix_layout(h2_matrix* A, const h2_tree* t, const std::vector<int32_t>& rank);
void matrix_alloc(h2_matrix* A, h2_precision prec);
std::unique_ptr<h2_matrix> matrix_clone_layout(const h2_matrix* A);

// HGEMV on tree-order column-major vectors (no permutation)
// nt_force (1, 2 or 4) fixes the matrix-core tile width (tests); 0: autotuned
void gemv_tree_f64(const h2_matrix* A, int nv, double alpha, const double* xt, int ldx,
                   double beta, double* yt, int ldy, hipStream_t s, int nt_force = 0);
void gemv_tree_f32(const h2_matrix* A, int nv, float alpha, const float* xt, int ldx,
                   float beta, float* yt, int ldy, hipStream_t s, int nt_force = 0);

// permutations between user and tree order (column-major, nv columns)
void gather_rows(const h2_tree* t, int nv, const double* x, int ldx, double* xt, int ldt,
                 hipStream_t s);
void scatter_rows(const h2_tree* t, int nv, double alpha, const double* yt, int ldt, double beta,
                  double* y, int ldy, hipStream_t s);
void gather_rows_f32(const h2_tree* t, int nv, const float* x, int ldx, float* xt, int ldt,
                     hipStream_t s);
void scatter_rows_f32(const h2_tree* t, int nv, float alpha, const float* yt, int ldt, float beta,
                      float* y, int ldy, hipStream_t s);

// counter-based Gaussian fill (splitmix64 + Box-Muller); see h2_build
uint64_t stream_key(uint64_t seed, uint32_t phase, uint32_t level, uint32_t round, uint32_t iter);
enum { PHASE_NORM = 1, PHASE_RANGE = 2, PHASE_PROBE = 5, PHASE_RESID = 6, PHASE_LOST = 8 };

}  // namespace h2
