// mlp_mfma.h -- wave-level inference of the 16-64-64-3 warm-start network
// on gfx950 matrix cores (v_mfma_f32_16x16x16_bf16): bf16 weights and
// bf16-rounded layer inputs, fp32 accumulation, fp32 bias and ReLU.
//
// Layers are computed transposed, H^T = W X^T: the A operand is a 16x16
// weight tile (rows = outputs, cols = inputs), the B operand holds 16
// contacts (cols) by 16 inputs (rows).  With the 16x16x16 layouts
//   A: lane l holds A[l%16][4(l/16) + i]      B: lane l holds B[4(l/16) + i][l%16]
//   D: lane l holds D[4(l/16) + i][l%16]      (i = 0..3)
// the accumulator of one layer (4 hidden units of one contact per lane) is
// exactly the B operand of the next, so hidden activations never leave
// registers.  Each wave runs 64 contacts as four tiles of 16.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sim_internal.h"

namespace rbs {

typedef short mfma_s4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t f2bf(float x) {
  // round to nearest even; inf/nan keep their class
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return u >> 16;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ mfma_s4 pack4(float a, float b, float c, float d) {
  mfma_s4 r;
  r.x = (short)f2bf(a);
  r.y = (short)f2bf(b);
  r.z = (short)f2bf(c);
  r.w = (short)f2bf(d);
  return r;
}

// Weight tile of a row-major bf16 matrix W[rows][cols] as the A operand:
// lane l reads W[r0 + l%16][c0 + 4(l/16) .. +3]; rows >= nrows read zero.
__device__ __forceinline__ mfma_s4 load_a_tile(const uint16_t* W, int cols, int nrows, int r0, int c0) {
  const int l = threadIdx.x & 63;
  const int r = r0 + (l & 15), c = c0 + 4 * (l >> 4);
  mfma_s4 v = {0, 0, 0, 0};
  if (r < nrows) {
    const uint2 u = *reinterpret_cast<const uint2*>(W + (long)r * cols + c);
    v.x = (short)(u.x & 0xffffu);
    v.y = (short)(u.x >> 16);
    v.z = (short)(u.y & 0xffffu);
    v.w = (short)(u.y >> 16);
  }
  return v;
}

__device__ __forceinline__ uint32_t bperm(uint32_t v, int src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}

// All 64 lanes must call this together.  x: the lane's 16 raw features
// (ignored when !valid).  y: the lane's 3 outputs.
__device__ inline void mlp_wave(const MlpParams& M, const float* x, bool valid, float* y) {
  const int l = threadIdx.x & 63;
  const int g = l >> 4, col = l & 15;
  // normalised, bf16-rounded features packed two per dword
  uint32_t zp[8];
#pragma unroll
  for (int p = 0; p < 8; p++) {
    float z0 = 0.f, z1 = 0.f;
    if (valid) {
      z0 = (x[2 * p] - M.mean[2 * p]) / fmaxf(M.stdv[2 * p], 1e-6f);
      z1 = (x[2 * p + 1] - M.mean[2 * p + 1]) / fmaxf(M.stdv[2 * p + 1], 1e-6f);
    }
    zp[p] = f2bf(z0) | (f2bf(z1) << 16);
  }
  // weight tiles are loaded where they are used (the caches serve the
  // repeats of the four contact tiles), so that few registers hold them
  float yt[4][3];
#pragma unroll
  for (int t = 0; t < 4; t++) {
    // B operand of layer 1: contact 16t + col, features 4g..4g+3
    const int src = 16 * t + col;
    uint32_t got[8];
#pragma unroll
    for (int p = 0; p < 8; p++) got[p] = bperm(zp[p], src);
    uint32_t d0 = g == 0 ? got[0] : g == 1 ? got[2] : g == 2 ? got[4] : got[6];
    uint32_t d1 = g == 0 ? got[1] : g == 1 ? got[3] : g == 2 ? got[5] : got[7];
    mfma_s4 xb;
    xb.x = (short)(d0 & 0xffffu);
    xb.y = (short)(d0 >> 16);
    xb.z = (short)(d1 & 0xffffu);
    xb.w = (short)(d1 >> 16);
    mfma_s4 h1[4], h2[4];
#pragma unroll
    for (int mb = 0; mb < 4; mb++) {
      const int r = 16 * mb + 4 * g;
      mfma_f4 acc = {M.b1[r], M.b1[r + 1], M.b1[r + 2], M.b1[r + 3]};
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(load_a_tile(M.w1, 16, 64, 16 * mb, 0), xb, acc, 0, 0, 0);
      h1[mb] = pack4(fmaxf(acc.x, 0.f), fmaxf(acc.y, 0.f), fmaxf(acc.z, 0.f), fmaxf(acc.w, 0.f));
    }
#pragma unroll
    for (int mb = 0; mb < 4; mb++) {
      const int r = 16 * mb + 4 * g;
      mfma_f4 acc = {M.b2[r], M.b2[r + 1], M.b2[r + 2], M.b2[r + 3]};
#pragma unroll
      for (int kb = 0; kb < 4; kb++)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(load_a_tile(M.w2, 64, 64, 16 * mb, 16 * kb), h1[kb], acc, 0,
                                                        0, 0);
      h2[mb] = pack4(fmaxf(acc.x, 0.f), fmaxf(acc.y, 0.f), fmaxf(acc.z, 0.f), fmaxf(acc.w, 0.f));
    }
    mfma_f4 acc = {g == 0 ? M.b3[0] : 0.f, g == 0 ? M.b3[1] : 0.f, g == 0 ? M.b3[2] : 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; kb++)
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(load_a_tile(M.w3, 64, 3, 0, 16 * kb), h2[kb], acc, 0, 0, 0);
    // outputs of contact 16t + col sit in lane col (rows 0..2 of the tile)
    yt[t][0] = acc.x;
    yt[t][1] = acc.y;
    yt[t][2] = acc.z;
  }
  // back to the owning lane: contact l is tile l/16, lane l%16
#pragma unroll
  for (int o = 0; o < 3; o++) {
    float v[4];
#pragma unroll
    for (int t = 0; t < 4; t++) v[t] = __uint_as_float(bperm(__float_as_uint(yt[t][o]), col));
    y[o] = g == 0 ? v[0] : g == 1 ? v[1] : g == 2 ? v[2] : v[3];
  }
}

}  // namespace rbs
