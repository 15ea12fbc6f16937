// Wave-level inference of the learned acceptance criterion's network
// (12 -> 64 -> 64 -> 1, ReLU) on the gfx950 matrix cores.
//
// Arithmetic: inputs, weights and hidden activations are rounded to BF16
// (round to nearest even) before every product; products accumulate in FP32
// (v_mfma_f32_16x16x16_bf16, exact BF16 x BF16 products); biases are FP32.
//
// Layout: the layers are computed transposed, H^T = W X^T, so that a layer's
// 16x16 output blocks are already the next layer's B operands.  For the
// 16x16x16 BF16 MFMA, lane l holds
//   A: row l%16, columns 4(l/16) .. 4(l/16)+3        (4 BF16)
//   B: rows 4(l/16) .. 4(l/16)+3, column l%16        (4 BF16)
//   D: rows 4(l/16) .. 4(l/16)+3, column l%16        (4 FP32)
// Rows of A are hidden units, columns of B are samples: a 16-sample tile
// needs 4 MFMAs for layer 1 (K = 16: 12 features + 4 zero columns) and 16 for
// layer 2 (K = 64 as 4 blocks); layer 3 is a dot product folded across the
// four lane groups.  Weights are read straight from their row-major BF16
// images (8-byte loads), biases and w3 as float4 per lane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "octgrav_internal.h"

namespace octgrav {

namespace dev {

typedef short v4s16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float(bf16_bits(f) << 16); }

__device__ __forceinline__ v4s16 pack4(float a, float b, float c, float d) {
  v4s16 r;
  r[0] = (short)bf16_bits(a);
  r[1] = (short)bf16_bits(b);
  r[2] = (short)bf16_bits(c);
  r[3] = (short)bf16_bits(d);
  return r;
}

__device__ __forceinline__ v4s16 load4(const uint16_t* p) {
  const uint2 u = *reinterpret_cast<const uint2*>(p);
  v4s16 r;
  r[0] = (short)(u.x & 0xFFFFu);
  r[1] = (short)(u.x >> 16);
  r[2] = (short)(u.y & 0xFFFFu);
  r[3] = (short)(u.y >> 16);
  return r;
}

// Pre-activations of one 16-sample tile t of the 64 staged samples
// (xs: LDS, BF16 bits [64][16]).  a1[mb][r] and a2[mb][r] are hidden unit
// 16 mb + 4 (l/16) + r of sample 16 t + l%16.  Returns that sample's output
// in every lane (after the fold, all four lane groups hold it).
__device__ __forceinline__ float mlp_tile(const uint8_t* __restrict__ pk,
                                          const uint16_t* xs, int t, int lane, v4f32* a1,
                                          v4f32* a2) {
  const uint16_t* w1 = reinterpret_cast<const uint16_t*>(pk + kPkW1);
  const uint16_t* w2 = reinterpret_cast<const uint16_t*>(pk + kPkW2);
  const float* b1 = reinterpret_cast<const float*>(pk + kPkB1);
  const float* b2 = reinterpret_cast<const float*>(pk + kPkB2);
  const float* w3 = reinterpret_cast<const float*>(pk + kPkW3);
  const int row = lane & 15, quad = lane >> 4;
  const v4s16 xb = load4(xs + (16 * t + row) * kMlpInPad + 4 * quad);
  v4s16 h1[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const float4 bb = *reinterpret_cast<const float4*>(b1 + 16 * mb + 4 * quad);
    v4f32 c = {bb.x, bb.y, bb.z, bb.w};
    const v4s16 a = load4(w1 + (16 * mb + row) * kMlpInPad + 4 * quad);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, xb, c, 0, 0, 0);
    a1[mb] = c;
    h1[mb] = pack4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
  }
  float s = 0.f;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const float4 bb = *reinterpret_cast<const float4*>(b2 + 16 * mb + 4 * quad);
    v4f32 c = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const v4s16 a = load4(w2 + (16 * mb + row) * kMlpH + 16 * kb + 4 * quad);
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, h1[kb], c, 0, 0, 0);
    }
    a2[mb] = c;
    const float4 ww = *reinterpret_cast<const float4*>(w3 + 16 * mb + 4 * quad);
    s += ww.x * bf16_round(fmaxf(c[0], 0.f));
    s += ww.y * bf16_round(fmaxf(c[1], 0.f));
    s += ww.z * bf16_round(fmaxf(c[2], 0.f));
    s += ww.w * bf16_round(fmaxf(c[3], 0.f));
  }
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s + *reinterpret_cast<const float*>(pk + kPkB3);
}

// Network output for the sample staged in LDS row `lane` (all 64 lanes must
// be active; rows of lanes without a sample may hold anything finite).
__device__ __forceinline__ float mlp_scores64(const uint8_t* __restrict__ pk, const uint16_t* xs,
                                              int lane) {
  float y = 0.f;
  v4f32 a1[4], a2[4];
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    const float s = mlp_tile(pk, xs, t, lane, a1, a2);
    if ((lane >> 4) == t) y = s;
  }
  return y;
}

// Stages one lane's 12 features as a BF16 row of 16 (4 zero columns).
__device__ __forceinline__ void mlp_stage(uint16_t* xs, int lane, const float* f) {
  uint32_t* row = reinterpret_cast<uint32_t*>(xs + lane * kMlpInPad);
#pragma unroll
  for (int k = 0; k < 6; ++k) row[k] = bf16_bits(f[2 * k]) | (bf16_bits(f[2 * k + 1]) << 16);
  row[6] = 0;
  row[7] = 0;
}

}  // namespace dev
}  // namespace octgrav
