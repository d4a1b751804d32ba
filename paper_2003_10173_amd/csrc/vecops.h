// Small device vector utilities used by the drivers (norms, scaling, fills).
#pragma once

#include <functional>

#include "internal.h"

namespace h2 {

// v[r] = Gaussian entry (tree row r, column col) of stream key, r < n, for
// `ncols` columns of a column-major array with leading dimension ld
void gauss_fill(uint64_t key, int n, int ncols, int col0, double* v, int ld, hipStream_t s);
// Euclidean norm of a device vector (synchronises the stream)
double nrm2(int n, const double* v, hipStream_t s);
// v *= a
void scal(int n, double a, double* v, hipStream_t s);
// y = a x + b y (column-major blocks of ncols columns)
void axpby(int n, int ncols, double a, const double* x, int ldx, double b, double* y, int ldy,
           hipStream_t s);

// Power method on a symmetric operator op(v, w): w = A v (device, n-vectors).
// Start vector: Gaussian stream (seed, phase, 0, 0, iteration), column 0.
// Stops when |nu - nu_prev| <= rel nu after at least min_it steps.
double power_norm_device(int n, const std::function<void(const double*, double*)>& op,
                         uint64_t seed, uint32_t iteration, double rel, int min_it, int max_it,
                         hipStream_t s, int* iters, int phase = PHASE_NORM, bool sqrt_out = false);

// Power iterations of several symmetric operators in lock step: each step
// enqueues every unfinished job's w = op(v), |w| and v = w / |w| on the
// device, then one copy of all norms to the host decides which jobs stop.
// op must enqueue on the stream it is given.  graph: after an eager first
// step (which sizes the operators' workspaces) the step's launch sequence is
// captured once per set of unfinished jobs and replayed.
struct PowerJob {
  int n = 0;
  std::function<void(const double*, double*, hipStream_t)> op;
  uint64_t seed = 1;
  uint32_t iteration = 0;
  int phase = PHASE_NORM;
  double rel = 1e-2;
  int min_it = 3, max_it = 30;
  bool sqrt_out = false;
  double result = 0;            // norm (or its square root with sqrt_out)
  int iters = 0;
  std::vector<double> history;  // the value after every step
};
// batch_op (optional, no graph): one call per step applies every unfinished
// job's operator, jobs[k] taking v[k] to w[k], instead of the per-job ops
using PowerBatchOp = std::function<void(const std::vector<int>& jobs,
                                        const std::vector<const double*>& v,
                                        const std::vector<double*>& w, hipStream_t)>;
void power_norm_multi(std::vector<PowerJob>& jobs, hipStream_t s, bool graph,
                      const PowerBatchOp* batch_op = nullptr);

}  // namespace h2
