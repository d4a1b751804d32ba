// Construction interface shared by h2_build and the Newton-Schulz driver.
#pragma once

#include <memory>

#include "internal.h"
#include "linalg.h"

namespace h2 {

struct PackedBatch;

// Operator to be compressed, applied to tree-ordered column-major blocks
// (ld = n): Y = A Omega.  `applies` counts columns.
struct Sampler {
  int64_t applies = 0;
  virtual ~Sampler() = default;
  virtual void apply(Ctx& c, int ncols, const double* om, double* y) = 0;
  // samplers of one problem of a batch served by one batched user callback
  virtual PackedBatch* batch() { return nullptr; }
  virtual int batch_index() const { return -1; }
};

// One product request of a phase: y (n x ncols) = S (om), tree order, ld n.
struct ApplyReq {
  Sampler* S;
  int ncols;
  const double* om;
  double* y;
};
// Serves every request; requests whose samplers belong to one PackedBatch
// are served by one call of its batched user callback.
void apply_requests(Ctx& c, const std::vector<ApplyReq>& reqs);

// The problems of h2_build_batched_packed: one h2_batched_sampler_fn over the
// packed layout (problem i owns user-ordered rows off[i] .. off[i+1] - 1),
// all requested problems sharing the column count of the call.
struct PackedBatch {
  h2_batched_sampler_fn fn = nullptr;
  void* ctx = nullptr;
  std::vector<const h2_tree*> trees;
  std::vector<int64_t> off;
  DevBuf om, y;
  int64_t calls = 0;
  // (problem index, ncols, om, y) per request, tree order
  void apply(Ctx& c, const std::vector<std::tuple<int, int, const double*, double*>>& reqs);
};

struct PackedSampler : Sampler {
  PackedBatch* B;
  int idx;
  PackedSampler(PackedBatch* b, int i) : B(b), idx(i) {}
  void apply(Ctx& c, int ncols, const double* om, double* y) override {
    B->apply(c, {{idx, ncols, om, y}});
    applies += ncols;
  }
  PackedBatch* batch() override { return B; }
  int batch_index() const override { return idx; }
};

// Wraps a user h2_sampler_fn (user ordering) with the tree permutation.
struct UserSampler : Sampler {
  const h2_tree* t;
  h2_sampler_fn fn;
  void* ctx;
  DevBuf buf;
  UserSampler(const h2_tree* t_, h2_sampler_fn f, void* c_) : t(t_), fn(f), ctx(c_) {}
  void apply(Ctx& c, int ncols, const double* om, double* y) override;
};

struct BuildParams {
  int rank_cap = 32;
  int oversample = 10;
  double tol = 1e-4;
  bool adaptive = true;
  int max_rounds = 16;
  uint64_t seed = 1;
  uint32_t iteration = 0;
  double norm = 0;        // > 0: use as ||A||_2; else estimate
  double norm_rel = 1e-2;
  const h2_mlp* mlp = nullptr;  // rank predictor for the first round (adaptive mode)
  // numerical-rank cut of the range basis, relative to the largest singular
  // value of the samples: above the sampler's rounding level
  double rank_cut = 1e-13;
  // basis rank cap of the recompression (0: rank_cap, which also sets the
  // sampling width rank_cap + oversample)
  int dest_cap = 0;
};

// Peeling on the weak partition + recompression into the strong H2 of `t`.
std::unique_ptr<h2_matrix> build_h2(const h2_tree* t, Sampler& S, const BuildParams& p, Ctx& c,
                                    h2_build_stats* st, bool* converged);

// Several independent problems built level-synchronously: every launch of a
// phase covers the blocks of all problems that have that level (the samplers
// are applied problem by problem).  Each problem's result equals its own
// build_h2 (the batched kernels treat every matrix independently).
struct BuildJob {
  const h2_tree* t = nullptr;
  Sampler* S = nullptr;
  BuildParams prm;
  h2_build_stats stats{};
  bool converged = true;
  std::unique_ptr<h2_matrix> out;
};
void build_h2_multi(std::vector<BuildJob>& jobs, Ctx& c);

}  // namespace h2
