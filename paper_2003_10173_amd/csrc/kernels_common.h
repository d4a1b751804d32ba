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

// DPP move of a double (both 32-bit halves); lanes whose row is outside
// ROW_MASK receive no defined value (the sums below never read them)
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// value of lane `lane` (wave-uniform) as a uniform double
__device__ inline double readlane_f64(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 64 lanes of a wave, returned to every lane.  Data-parallel
// moves (no LDS traffic): pairs and quads within each row of 16 lanes, the
// half-row and row mirrors complete the row sums, two row broadcasts
// accumulate the four rows into lane 63 (rows left out of a broadcast hold
// partial values that lane 63 never reads), which is read back as a uniform
// value.  Every lane of the wave must be active.
template <>
__device__ inline double wave_sum<double>(double v) {
  v += dpp_f64<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_f64<0x140, 0xf>(v);  // row_mirror
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return readlane_f64(v, 63);
}

// K independent wave sums at once, stage by stage, so that the data moves of
// the K reductions overlap (same order of additions as wave_sum)
template <int K>
__device__ inline void wave_sum_n(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f64<0xB1, 0xf>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f64<0x4E, 0xf>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f64<0x141, 0xf>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f64<0x140, 0xf>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f64<0x142, 0xa>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f64<0x143, 0xc>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = readlane_f64(v[k], 63);
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
