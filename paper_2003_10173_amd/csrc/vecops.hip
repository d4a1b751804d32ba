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

double power_norm_device(int n, const std::function<void(const double*, double*)>& op,
                         uint64_t seed, uint32_t iteration, double rel, int min_it, int max_it,
                         hipStream_t s, int* iters, int phase, bool sqrt_out) {
  DevBuf vb((size_t)2 * n * sizeof(double));
  double* v = vb.as<double>();
  double* w = v + n;
  gauss_fill(stream_key(seed, phase, 0, 0, iteration), n, 1, 0, v, n, s);
  double nv = nrm2(n, v, s);
  H2_CHECK(std::isfinite(nv) && nv > 0, H2_ENUMERIC, "power method start vector is degenerate");
  scal(n, 1.0 / nv, v, s);
  double prev = -1.0, val = 0.0;
  int it = 0;
  for (it = 1; it <= max_it; ++it) {
    op(v, w);
    double nu = nrm2(n, w, s);
    H2_CHECK(std::isfinite(nu), H2_ENUMERIC, "power method met a non-finite value");
    if (nu == 0.0) { val = 0.0; break; }
    H2_HIP(hipMemcpyAsync(v, w, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    scal(n, 1.0 / nu, v, s);
    val = sqrt_out ? std::sqrt(nu) : nu;
    if (prev >= 0 && it >= min_it && std::fabs(val - prev) <= rel * val) break;
    prev = val;
  }
  if (iters) *iters = std::min(it, max_it);
  return val;
}

}  // namespace h2
