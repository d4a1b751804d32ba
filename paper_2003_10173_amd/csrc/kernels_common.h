// Device helpers shared by the library's kernels: precision conversions,
// block reductions and the counter-based Gaussian generator.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2 {

// BF16 storage as raw bits; conversion FP32 -> BF16 rounds to nearest even.
struct bf16_t {
  uint16_t bits;
};

__host__ __device__ inline float bf16_to_float(bf16_t b) {
  union { uint32_t u; float f; } c;
  c.u = (uint32_t)b.bits << 16;
  return c.f;
}
__host__ __device__ inline bf16_t float_to_bf16(float f) {
  union { uint32_t u; float f; } c;
  c.f = f;
  uint32_t u = c.u;
  if ((u & 0x7f800000u) == 0x7f800000u) {  // Inf / NaN: keep, quiet NaN
    bf16_t r;
    r.bits = (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    return r;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  bf16_t r;
  r.bits = (uint16_t)(u >> 16);
  return r;
}

template <class V> __device__ inline V to_acc(double x) { return (V)x; }
template <class V> __device__ inline V to_acc(float x) { return (V)x; }
template <class V> __device__ inline V to_acc(bf16_t x) { return (V)bf16_to_float(x); }

__device__ inline double to_double(double x) { return x; }
__device__ inline double to_double(float x) { return (double)x; }
__device__ inline double to_double(bf16_t x) { return (double)bf16_to_float(x); }

template <class T> __device__ inline T from_double(double x);
template <> __device__ inline double from_double<double>(double x) { return x; }
template <> __device__ inline float from_double<float>(double x) { return (float)x; }
template <> __device__ inline bf16_t from_double<bf16_t>(double x) { return float_to_bf16((float)x); }

// ------------------------------------------------------------------ splitmix64
// n-th output of the splitmix64 stream with state `key` (Steele, Lea, Flood 2014)
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;

// Gaussian entry (tree row r, column j) of the stream `key`: outputs
// n = 2 (r 2^16 + j) + 1 and n + 1, uniforms in (0, 1], Box-Muller.
__device__ inline double gauss_entry(uint64_t key, uint64_t r, uint64_t j) {
  const uint64_t n = 2ull * ((r << 16) + j) + 1ull;
  const uint64_t x1 = mix64(key + n * SM_GAMMA);
  const uint64_t x2 = mix64(key + (n + 1ull) * SM_GAMMA);
  const double scale = 1.0 / 9007199254740992.0;  // 2^-53
  const double u1 = ((double)(x1 >> 11) + 1.0) * scale;
  const double u2 = ((double)(x2 >> 11) + 1.0) * scale;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// ------------------------------------------------------------------ reductions
template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <class T>
__device__ inline T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = v > o ? v : o;
  }
  return v;
}

// block-wide sum for blockDim.x == 256 (4 waves); `red` has >= 4 entries
template <class T>
__device__ inline T block_sum256(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T s = red[0] + red[1] + red[2] + red[3];
  return s;
}

}  // namespace h2
