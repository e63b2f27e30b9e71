// Learned bucket classifier: BF16 parameter handling, the 8-64-64-2 network
// evaluated with FP32 accumulation, and the bucket features.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfft_device.hpp"

namespace sfft {

constexpr int kMlpIn = 8, kMlpH = 64, kMlpOut = 2;
constexpr int kMlpParams = 4866;
// offsets of W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [2][64], b3 [2]
constexpr int kW1 = 0, kB1 = 512, kW2 = 576, kB2 = 4672, kW3 = 4736, kB3 = 4864;

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}

// Round to nearest BF16, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_round(float f) { return bf16_to_f32(f32_to_bf16(f)); }

// Parameters (BF16, global) into LDS as FP32; all threads of the work-group.
__device__ inline void mlp_load(const uint16_t* __restrict__ w, float* wl) {
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) wl[i] = bf16_to_f32(w[i]);
  __syncthreads();
}

// Logits of one input row (already BF16-rounded), one thread, FP32 accumulation.
__device__ inline void mlp_logits(const float* W, const float* x, float* z) {
  float h1[kMlpH];
#pragma unroll
  for (int o = 0; o < kMlpH; ++o) {
    float a = W[kB1 + o];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) a += W[kW1 + o * kMlpIn + i] * x[i];
    h1[o] = a > 0.f ? a : 0.f;
  }
  float z0 = W[kB3], z1 = W[kB3 + 1];
  for (int o = 0; o < kMlpH; ++o) {
    float a = W[kB2 + o];
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) a += W[kW2 + o * kMlpH + i] * h1[i];
    const float h = a > 0.f ? a : 0.f;
    z0 += W[kW3 + o] * h;
    z1 += W[kW3 + kMlpH + o] * h;
  }
  z[0] = z0;
  z[1] = z1;
}

// Probability of class 1 ("one mode"): 1 / (1 + exp(z0 - z1)).
__device__ inline float mlp_prob(const float* W, const float* x) {
  float z[2];
  mlp_logits(W, x, z);
  return 1.f / (1.f + expf(z[0] - z[1]));
}

}  // namespace sfft
