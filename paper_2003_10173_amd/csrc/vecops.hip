// Device vector utilities: counter-based Gaussian fills, norms, scaling and
// the power method for 2-norm estimates (Sec. 3.2: p-norms by the power
// method, stopped once the value has settled to two significant digits).
#include <cmath>

#include "kernels_common.h"
#include "vecops.h"

namespace h2 {

uint64_t stream_key(uint64_t seed, uint32_t phase, uint32_t level, uint32_t round, uint32_t iter) {
  const uint64_t tag = ((uint64_t)phase << 56) | ((uint64_t)level << 48) | ((uint64_t)round << 32) |
                       (uint64_t)iter;
  return mix64(mix64(seed + SM_GAMMA) ^ tag);
}

__global__ void k_gauss_fill(uint64_t key, int n, int ncols, int col0, double* __restrict__ v,
                             int ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * ncols) return;
  const int r = (int)(e % n), j = (int)(e / n);
  v[(size_t)j * ld + r] = gauss_entry(key, (uint64_t)r, (uint64_t)(col0 + j));
}

void gauss_fill(uint64_t key, int n, int ncols, int col0, double* v, int ld, hipStream_t s) {
  const int64_t tot = (int64_t)n * ncols;
  if (tot == 0) return;
  k_gauss_fill<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(key, n, ncols, col0, v, ld);
  H2_LAUNCH_CHECK();
}

// single-block sum of squares (deterministic order), result in out[0]
__global__ __launch_bounds__(1024) void k_sumsq(int n, const double* __restrict__ v,
                                                double* __restrict__ out) {
  __shared__ double red[16];
  double s = 0;
  for (int i = threadIdx.x; i < n; i += 1024) s += v[i] * v[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < 16; ++w) t += red[w];
    out[0] = t;
  }
}

__global__ void k_scal(int n, double a, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] *= a;
}

__global__ void k_axpby(int n, int ncols, double a, const double* __restrict__ x, int ldx, double b,
                        double* __restrict__ y, int ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * ncols) return;
  const int r = (int)(e % n), j = (int)(e / n);
  double* yp = y + (size_t)j * ldy + r;
  const double xv = a * x[(size_t)j * ldx + r];
  *yp = b == 0.0 ? xv : xv + b * *yp;
}

double nrm2(int n, const double* v, hipStream_t s) {
  DevBuf out(sizeof(double));
  k_sumsq<<<1, 1024, 0, s>>>(n, v, out.as<double>());
  H2_LAUNCH_CHECK();
  double h = 0;
  H2_HIP(hipMemcpyAsync(&h, out.p, sizeof(double), hipMemcpyDeviceToHost, s));
  H2_HIP(hipStreamSynchronize(s));
  return std::sqrt(h);
}

void scal(int n, double a, double* v, hipStream_t s) {
  if (n == 0) return;
  k_scal<<<(n + 255) / 256, 256, 0, s>>>(n, a, v);
  H2_LAUNCH_CHECK();
}

void axpby(int n, int ncols, double a, const double* x, int ldx, double b, double* y, int ldy,
           hipStream_t s) {
  const int64_t tot = (int64_t)n * ncols;
  if (tot == 0) return;
  k_axpby<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(n, ncols, a, x, ldx, b, y, ldy);
  H2_LAUNCH_CHECK();
}

// v = w / sqrt(ss[0]) (v = 0 when ss[0] is zero)
__global__ void k_normalize(int n, const double* __restrict__ w, const double* __restrict__ ss,
                            double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double nrm = sqrt(ss[0]);
  v[i] = nrm > 0.0 ? w[i] / nrm : 0.0;
}

namespace {
// device buffers of one job: v, w and the sum of squares of w
struct PowerBufs {
  DevBuf vw;
  double* v = nullptr;
  double* w = nullptr;
};

void enqueue_step(PowerJob& J, PowerBufs& B, double* ss, hipStream_t s) {
  J.op(B.v, B.w, s);
  k_sumsq<<<1, 1024, 0, s>>>(J.n, B.w, ss);
  k_normalize<<<(J.n + 255) / 256, 256, 0, s>>>(J.n, B.w, ss, B.v);
}
}  // namespace

void power_norm_multi(std::vector<PowerJob>& jobs, hipStream_t s, bool graph,
                      const PowerBatchOp* batch_op) {
  if (batch_op) graph = false;
  const int nj = (int)jobs.size();
  if (nj == 0) return;
  std::vector<PowerBufs> B(nj);
  DevBuf ssb((size_t)nj * sizeof(double));
  double* ss = ssb.as<double>();
  std::vector<double> hs(nj);
  // start vectors: Gaussian, normalised
  for (int j = 0; j < nj; ++j) {
    PowerJob& J = jobs[j];
    B[j].vw.alloc((size_t)2 * J.n * sizeof(double));
    B[j].v = B[j].vw.as<double>();
    B[j].w = B[j].v + J.n;
    gauss_fill(stream_key(J.seed, J.phase, 0, 0, J.iteration), J.n, 1, 0, B[j].v, J.n, s);
    k_sumsq<<<1, 1024, 0, s>>>(J.n, B[j].v, ss + j);
    k_normalize<<<(J.n + 255) / 256, 256, 0, s>>>(J.n, B[j].v, ss + j, B[j].v);
    H2_LAUNCH_CHECK();
    J.result = 0;
    J.iters = 0;
    J.history.clear();
  }
  H2_HIP(hipMemcpyAsync(hs.data(), ss, nj * sizeof(double), hipMemcpyDeviceToHost, s));
  H2_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < nj; ++j)
    H2_CHECK(std::isfinite(hs[j]) && hs[j] > 0, H2_ENUMERIC, "power method start vector is degenerate");
  std::vector<char> active(nj, 1);
  std::vector<double> prev(nj, -1.0);
  // the captured step of the current active set (re-captured when it changes)
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<char> exec_set;
  auto drop_graph = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  };
  try {
    for (int it = 1;; ++it) {
      bool any = false;
      for (int j = 0; j < nj; ++j) any = any || active[j];
      if (!any) break;
      // the first step runs eagerly (it sizes the operators' workspaces)
      const bool use_graph = graph && it >= 2;
      if (use_graph) {
        if (!exec || exec_set != active) {
          drop_graph();
          if (!cap) H2_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
          hipGraph_t g = nullptr;
          H2_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
          try {
            for (int j = 0; j < nj; ++j)
              if (active[j]) enqueue_step(jobs[j], B[j], ss + j, cap);
          } catch (...) {
            (void)hipStreamEndCapture(cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
          }
          H2_HIP(hipStreamEndCapture(cap, &g));
          const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          H2_HIP(e);
          exec_set = active;
        }
        H2_HIP(hipGraphLaunch(exec, s));
      } else if (batch_op) {
        std::vector<int> ids;
        std::vector<const double*> vs;
        std::vector<double*> ws;
        for (int j = 0; j < nj; ++j)
          if (active[j]) {
            ids.push_back(j);
            vs.push_back(B[j].v);
            ws.push_back(B[j].w);
          }
        (*batch_op)(ids, vs, ws, s);
        for (int j : ids) {
          k_sumsq<<<1, 1024, 0, s>>>(jobs[j].n, B[j].w, ss + j);
          k_normalize<<<(jobs[j].n + 255) / 256, 256, 0, s>>>(jobs[j].n, B[j].w, ss + j, B[j].v);
        }
        H2_LAUNCH_CHECK();
      } else {
        for (int j = 0; j < nj; ++j)
          if (active[j]) enqueue_step(jobs[j], B[j], ss + j, s);
        H2_LAUNCH_CHECK();
      }
      H2_HIP(hipMemcpyAsync(hs.data(), ss, nj * sizeof(double), hipMemcpyDeviceToHost, s));
      H2_HIP(hipStreamSynchronize(s));
      for (int j = 0; j < nj; ++j) {
        if (!active[j]) continue;
        PowerJob& J = jobs[j];
        const double nu = std::sqrt(hs[j]);
        H2_CHECK(std::isfinite(nu), H2_ENUMERIC, "power method met a non-finite value");
        J.iters = it;
        if (nu == 0.0) {
          J.result = 0.0;
          active[j] = 0;
          continue;
        }
        const double val = J.sqrt_out ? std::sqrt(nu) : nu;
        J.result = val;
        J.history.push_back(val);
        if ((prev[j] >= 0 && it >= J.min_it && std::fabs(val - prev[j]) <= J.rel * val) ||
            it >= J.max_it)
          active[j] = 0;
        prev[j] = val;
      }
    }
  } catch (...) {
    drop_graph();
    if (cap) (void)hipStreamDestroy(cap);
    throw;
  }
  drop_graph();
  if (cap) H2_HIP(hipStreamDestroy(cap));
}

double power_norm_device(int n, const std::function<void(const double*, double*)>& op,
                         uint64_t seed, uint32_t iteration, double rel, int min_it, int max_it,
                         hipStream_t s, int* iters, int phase, bool sqrt_out) {
  std::vector<PowerJob> jobs(1);
  PowerJob& J = jobs[0];
  J.n = n;
  J.op = [&](const double* v, double* w, hipStream_t) { op(v, w); };
  J.seed = seed;
  J.iteration = iteration;
  J.phase = phase;
  J.rel = rel;
  J.min_it = min_it;
  J.max_it = max_it;
  J.sqrt_out = sqrt_out;
  power_norm_multi(jobs, s, false);
  if (iters) *iters = J.iters;
  return J.result;
}

}  // namespace h2
