// mlp_infer.h -- per-contact inference of the 16-64-64-3 warm-start network
// inside the step kernel: bf16 weights and bf16-rounded layer inputs, fp32
// accumulation, fp32 bias and ReLU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sim_internal.h"

namespace rbs {

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to the nearest bf16 (ties to even), returned as float.
__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

__device__ inline void mlp_contact(const MlpParams& M, const float* x, float* y) {
  float z0[16];
#pragma unroll
  for (int i = 0; i < 16; i++) z0[i] = bf16_round((x[i] - M.mean[i]) / fmaxf(M.stdv[i], 1e-6f));
  float h1[64];
  for (int o = 0; o < 64; o++) {
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 16; i++) s += bf16_to_f(M.w1[16 * o + i]) * z0[i];
    s += M.b1[o];
    h1[o] = bf16_round(fmaxf(s, 0.f));
  }
  float h2[64];
  for (int o = 0; o < 64; o++) {
    float s = 0.f;
    for (int i = 0; i < 64; i++) s += bf16_to_f(M.w2[64 * o + i]) * h1[i];
    s += M.b2[o];
    h2[o] = bf16_round(fmaxf(s, 0.f));
  }
  for (int o = 0; o < 3; o++) {
    float s = 0.f;
    for (int i = 0; i < 64; i++) s += bf16_to_f(M.w3[64 * o + i]) * h2[i];
    y[o] = s + M.b3[o];
  }
}

}  // namespace rbs
