// Learned first-round sample counts: a 16 -> 64 -> 64 -> 1 ReLU network that
// predicts log(1 + sample columns a sibling block needs) from its geometry
// and the singular-value decay of its parent block (features listed in h2.h).  The
// products use BF16 copies of the weights (round to nearest even from the
// FP32 masters) with FP32 inputs, activations and accumulation; training is
// mean-squared error with Adam on the FP32 masters.
//
// Packed parameters (FP32): W1 64x16 row-major, b1 64, W2 64x64 row-major,
// b2 64, W3 64, b3 1.
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>

#include "internal.h"
#include "kernels_common.h"
#include "linalg.h"
#include "mlp.h"

struct h2_mlp {
  h2::DevBuf master, m, v, wb, grad, loss;
  int64_t step = 0;
};

namespace h2 {

h2_status guarded_status(const std::function<void()>& f);

constexpr int NF = H2_MLP_FEATURES, NH = H2_MLP_HIDDEN;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == H2_MLP_PARAMS, "packed parameter count");

__device__ inline bool is_weight(int i) {
  return i < OFF_B1 || (i >= OFF_W2 && i < OFF_B2) || (i >= OFF_W3 && i < OFF_B3);
}

// effective parameters in LDS: BF16 weights widened to FP32, FP32 biases
__device__ inline void load_params(float* P, const float* __restrict__ master,
                                   const uint16_t* __restrict__ wb) {
  for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) {
    bf16_t b;
    b.bits = wb[i];
    P[i] = is_weight(i) ? bf16_to_float(b) : master[i];
  }
}

__global__ __launch_bounds__(256) void k_mlp_fwd(int batch, const float* __restrict__ X,
                                                 const float* __restrict__ master,
                                                 const uint16_t* __restrict__ wb,
                                                 float* __restrict__ y) {
  __shared__ float P[NPARAM];
  load_params(P, master, wb);
  __syncthreads();
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= batch) return;
  float x[NF], h1[NH];
#pragma unroll
  for (int f = 0; f < NF; ++f) x[f] = X[(size_t)row * NF + f];
#pragma unroll 4
  for (int j = 0; j < NH; ++j) {
    float a = P[OFF_B1 + j];
#pragma unroll
    for (int f = 0; f < NF; ++f) a += P[OFF_W1 + j * NF + f] * x[f];
    h1[j] = fmaxf(a, 0.0f);
  }
  float out = P[OFF_B3];
  for (int j = 0; j < NH; ++j) {
    float a = P[OFF_B2 + j];
#pragma unroll
    for (int i = 0; i < NH; ++i) a += P[OFF_W2 + j * NH + i] * h1[i];
    out += P[OFF_W3 + j] * fmaxf(a, 0.0f);
  }
  y[row] = out;
}

// gradient of the mean squared error over `batch` rows, accumulated into grad
// (NPARAM) and loss (1); one workgroup per 128 rows
constexpr int GR = 128;
__global__ __launch_bounds__(256) void k_mlp_grad(int batch, const float* __restrict__ X,
                                                  const float* __restrict__ T,
                                                  const float* __restrict__ master,
                                                  const uint16_t* __restrict__ wb,
                                                  float* __restrict__ grad,
                                                  float* __restrict__ loss) {
  __shared__ float P[NPARAM];
  __shared__ float H1[GR][NH + 1];
  __shared__ float H2[GR][NH + 1];   // h2, later dz1
  __shared__ float DZ2[GR][NH + 1];
  __shared__ float XS[GR][NF + 1];
  __shared__ float DY[GR];
  __shared__ float red[256];
  load_params(P, master, wb);
  __syncthreads();
  const int tid = threadIdx.x;
  const int row = blockIdx.x * GR + tid;
  float lsum = 0.0f;
  if (tid < GR) {
    if (row < batch) {
      float x[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        x[f] = X[(size_t)row * NF + f];
        XS[tid][f] = x[f];
      }
      for (int j = 0; j < NH; ++j) {
        float a = P[OFF_B1 + j];
#pragma unroll
        for (int f = 0; f < NF; ++f) a += P[OFF_W1 + j * NF + f] * x[f];
        H1[tid][j] = fmaxf(a, 0.0f);
      }
      float out = P[OFF_B3];
      for (int j = 0; j < NH; ++j) {
        float a = P[OFF_B2 + j];
        for (int i = 0; i < NH; ++i) a += P[OFF_W2 + j * NH + i] * H1[tid][i];
        const float h = fmaxf(a, 0.0f);
        H2[tid][j] = h;
        out += P[OFF_W3 + j] * h;
      }
      const float d = out - T[row];
      lsum = d * d / (float)batch;
      const float dy = 2.0f * d / (float)batch;
      DY[tid] = dy;
      for (int j = 0; j < NH; ++j) DZ2[tid][j] = H2[tid][j] > 0.0f ? dy * P[OFF_W3 + j] : 0.0f;
    } else {
      DY[tid] = 0.0f;
      for (int j = 0; j < NH; ++j) { H1[tid][j] = 0.0f; H2[tid][j] = 0.0f; DZ2[tid][j] = 0.0f; }
      for (int f = 0; f < NF; ++f) XS[tid][f] = 0.0f;
    }
  }
  red[tid] = lsum;
  __syncthreads();
  // W3, b3, W2, b2
  if (tid < NH) {
    float a = 0.0f;
    for (int r = 0; r < GR; ++r) a += DY[r] * H2[r][tid];
    atomicAdd(&grad[OFF_W3 + tid], a);
  } else if (tid == NH) {
    float a = 0.0f;
    for (int r = 0; r < GR; ++r) a += DY[r];
    atomicAdd(&grad[OFF_B3], a);
  } else if (tid >= 128 && tid < 128 + NH) {
    const int j = tid - 128;
    float a = 0.0f;
    for (int r = 0; r < GR; ++r) a += DZ2[r][j];
    atomicAdd(&grad[OFF_B2 + j], a);
  }
  for (int e = tid; e < NH * NH; e += 256) {
    const int j = e / NH, i = e % NH;
    float a = 0.0f;
    for (int r = 0; r < GR; ++r) a += DZ2[r][j] * H1[r][i];
    atomicAdd(&grad[OFF_W2 + e], a);
  }
  __syncthreads();
  // dz1 = (W2^T dz2) masked by h1 > 0, into the h2 space
  if (tid < GR) {
    for (int i = 0; i < NH; ++i) {
      float a = 0.0f;
      for (int j = 0; j < NH; ++j) a += DZ2[tid][j] * P[OFF_W2 + j * NH + i];
      H2[tid][i] = H1[tid][i] > 0.0f ? a : 0.0f;
    }
  }
  __syncthreads();
  for (int e = tid; e < NH * NF; e += 256) {
    const int i = e / NF, f = e % NF;
    float a = 0.0f;
    for (int r = 0; r < GR; ++r) a += H2[r][i] * XS[r][f];
    atomicAdd(&grad[OFF_W1 + e], a);
  }
  if (tid < NH) {
    float a = 0.0f;
    for (int r = 0; r < GR; ++r) a += H2[r][tid];
    atomicAdd(&grad[OFF_B1 + tid], a);
  }
  // loss
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) atomicAdd(loss, red[0]);
}

__global__ void k_mlp_zero(float* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

__global__ void k_mlp_refresh(const float* __restrict__ master, uint16_t* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NPARAM) wb[i] = float_to_bf16(master[i]).bits;
}

__global__ void k_mlp_adam(float* __restrict__ master, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ grad, uint16_t* __restrict__ wb, float lr,
                           float bc1, float bc2, float beta1, float beta2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const float g = grad[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * g;
  const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float w = master[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  master[i] = w;
  wb[i] = float_to_bf16(w).bits;
}

void mlp_forward(const h2_mlp* M, int batch, const float* X, float* y, hipStream_t s) {
  if (batch <= 0) return;
  k_mlp_fwd<<<(unsigned)((batch + 255) / 256), 256, 0, s>>>(batch, X, M->master.as<float>(),
                                                            M->wb.as<uint16_t>(), y);
  H2_LAUNCH_CHECK();
}

static void mlp_gradient(const h2_mlp* M, int batch, const float* X, const float* T, float* grad,
                         float* loss, hipStream_t s) {
  k_mlp_zero<<<(NPARAM + 255) / 256, 256, 0, s>>>(grad, NPARAM);
  k_mlp_zero<<<1, 256, 0, s>>>(loss, 1);
  if (batch > 0)
    k_mlp_grad<<<(unsigned)((batch + GR - 1) / GR), 256, 0, s>>>(
        batch, X, T, M->master.as<float>(), M->wb.as<uint16_t>(), grad, loss);
  H2_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ training records
namespace {
struct Records {
  std::mutex mu;
  bool on = false;
  std::vector<float> feats, targets;
};
Records& recs() {
  static Records r;
  return r;
}
}  // namespace

bool records_on() { return recs().on; }
void records_add(const std::vector<float>& feats, const std::vector<float>& targets) {
  Records& R = recs();
  std::lock_guard<std::mutex> g(R.mu);
  if (!R.on) return;
  R.feats.insert(R.feats.end(), feats.begin(), feats.end());
  R.targets.insert(R.targets.end(), targets.begin(), targets.end());
}

}  // namespace h2

using namespace h2;

extern "C" {

h2_status h2_mlp_create(const float* params_host, h2_mlp** out) {
  return guarded_status([&] {
    H2_CHECK(params_host && out, H2_EINVAL, "null argument");
    for (int i = 0; i < NPARAM; ++i)
      H2_CHECK(std::isfinite(params_host[i]), H2_EINVAL, "non-finite parameter");
    auto M = std::make_unique<h2_mlp>();
    M->master.alloc(NPARAM * sizeof(float));
    M->m.alloc(NPARAM * sizeof(float));
    M->v.alloc(NPARAM * sizeof(float));
    M->grad.alloc(NPARAM * sizeof(float));
    M->loss.alloc(sizeof(float));
    M->wb.alloc(NPARAM * sizeof(uint16_t));
    H2_HIP(hipMemcpy(M->master.p, params_host, NPARAM * sizeof(float), hipMemcpyHostToDevice));
    H2_HIP(hipMemset(M->m.p, 0, NPARAM * sizeof(float)));
    H2_HIP(hipMemset(M->v.p, 0, NPARAM * sizeof(float)));
    k_mlp_refresh<<<(NPARAM + 255) / 256, 256>>>(M->master.as<float>(), M->wb.as<uint16_t>());
    H2_LAUNCH_CHECK();
    H2_HIP(hipDeviceSynchronize());
    *out = M.release();
  });
}

h2_status h2_mlp_params(const h2_mlp* M, float* params_host) {
  return guarded_status([&] {
    H2_CHECK(M && params_host, H2_EINVAL, "null argument");
    H2_HIP(hipDeviceSynchronize());
    H2_HIP(hipMemcpy(params_host, M->master.p, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  });
}

h2_status h2_mlp_forward(const h2_mlp* M, int batch, const float* X, float* y, hipStream_t s) {
  return guarded_status([&] {
    H2_CHECK(M && batch >= 0 && (batch == 0 || (X && y)), H2_EINVAL, "bad arguments");
    mlp_forward(M, batch, X, y, s);
  });
}

h2_status h2_mlp_gradient(const h2_mlp* M, int batch, const float* X, const float* target,
                          float* grad, float* loss, hipStream_t s) {
  return guarded_status([&] {
    H2_CHECK(M && batch >= 0 && grad && loss && (batch == 0 || (X && target)), H2_EINVAL,
             "bad arguments");
    mlp_gradient(M, batch, X, target, grad, loss, s);
  });
}

h2_status h2_mlp_train_step(h2_mlp* M, int batch, const float* X, const float* target, float lr,
                            hipStream_t s) {
  return guarded_status([&] {
    H2_CHECK(M && batch >= 1 && X && target && lr > 0, H2_EINVAL, "bad arguments");
    mlp_gradient(M, batch, X, target, M->grad.as<float>(), M->loss.as<float>(), s);
    M->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)M->step));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)M->step));
    k_mlp_adam<<<(NPARAM + 255) / 256, 256, 0, s>>>(M->master.as<float>(), M->m.as<float>(),
                                                    M->v.as<float>(), M->grad.as<float>(),
                                                    M->wb.as<uint16_t>(), lr, bc1, bc2, b1, b2,
                                                    1e-8f);
    H2_LAUNCH_CHECK();
  });
}

h2_status h2_mlp_last_loss(const h2_mlp* M, float* loss_host) {
  return guarded_status([&] {
    H2_CHECK(M && loss_host, H2_EINVAL, "null argument");
    H2_HIP(hipDeviceSynchronize());
    H2_HIP(hipMemcpy(loss_host, M->loss.p, sizeof(float), hipMemcpyDeviceToHost));
  });
}

void h2_mlp_destroy(h2_mlp* M) { delete M; }

h2_status h2_records_enable(int on) {
  return guarded_status([&] {
    Records& R = recs();
    std::lock_guard<std::mutex> g(R.mu);
    R.on = on != 0;
    R.feats.clear();
    R.targets.clear();
  });
}

h2_status h2_records_read(int64_t* count, float* features, float* targets) {
  return guarded_status([&] {
    H2_CHECK(count, H2_EINVAL, "null argument");
    Records& R = recs();
    std::lock_guard<std::mutex> g(R.mu);
    *count = (int64_t)R.targets.size();
    if (features) std::memcpy(features, R.feats.data(), R.feats.size() * sizeof(float));
    if (targets) std::memcpy(targets, R.targets.data(), R.targets.size() * sizeof(float));
  });
}

}  // extern "C"
