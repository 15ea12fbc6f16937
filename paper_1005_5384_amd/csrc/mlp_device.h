// Wave-level inference of the learned acceptance criterion's network
// (12 -> 64 -> 64 -> 1, ReLU) on the gfx950 matrix cores.
//
// Arithmetic: inputs, weights and hidden activations are rounded to BF16
// (round to nearest even) before every product; products accumulate in FP32
// (exact BF16 x BF16 products on the matrix cores); biases are FP32.
//
// Layout: the layers are computed transposed, H^T = W X^T, so that a layer's
// 16x16 output blocks are already the next layer's B operands.  For the
// 16x16x16 BF16 MFMA, lane l holds
//   A: row l%16, columns 4(l/16) .. 4(l/16)+3        (4 BF16)
//   B: rows 4(l/16) .. 4(l/16)+3, column l%16        (4 BF16)
//   D: rows 4(l/16) .. 4(l/16)+3, column l%16        (4 FP32)
// and for the 16x16x32 BF16 MFMA (gfx950) the same with 8 consecutive
// columns / rows 8(l/16) .. 8(l/16)+7.  Rows of A are hidden units, columns
// of B are samples.  Layer 1 (K = 16: 12 features + 4 zero columns) takes 4
// 16x16x16 MFMAs per 16-sample tile.  Layer 2 (K = 64) takes 8 16x16x32
// MFMAs: its B operand for K block q is the lane's two layer-1 output
// blocks 2q and 2q+1 side by side, i.e. the contraction index runs over the
// hidden units in the order 16(2q) + 4(l/16) + 0..3, 16(2q+1) + 4(l/16) +
// 0..3; the A operand reads W2's columns in that same order (two 8-byte
// loads per lane).  Layer 3 is two more 16x16x32 MFMAs whose A operand
// repeats w3 in all 16 rows, so every lane receives the output of its own
// column (sample) without a shuffle.  Biases are read as float4 per lane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "octgrav_internal.h"

namespace octgrav {

namespace dev {

typedef short v4s16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float(bf16_bits(f) << 16); }

typedef float v2f32 __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf16 __attribute__((ext_vector_type(2)));

// Two FP32 values to packed BF16 (round to nearest even; one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  const v2f32 x = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, v2bf16));
}

__device__ __forceinline__ v4s16 load4(const uint16_t* p) {
  return __builtin_bit_cast(v4s16, *reinterpret_cast<const uint2*>(p));
}

typedef short v2s16 __attribute__((ext_vector_type(2)));

// ReLU of two packed BF16 values: as 16-bit integers, negative BF16 values
// (and -0) are negative, so a signed max with 0 clears exactly them
// (relu(bf16(x)) == bf16(relu(x))).  One v_pk_max_i16.
__device__ __forceinline__ uint32_t relu_pk(uint32_t h) {
  const v2s16 z = {0, 0};
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(v2s16, h), z));
}

// Where the network's weights are read from: the packed image in global
// memory (row strides 16 / 64) or a copy in LDS with padded rows.
struct MlpView {
  const uint16_t* w1;  // BF16 [64][w1s], 12 used columns + zeros
  const uint16_t* w2;  // BF16 [64][w2s]
  const float* b1;
  const float* b2;
  const uint16_t* w3;  // BF16 [64]
  float b3;
  int w1s, w2s;
};

__device__ __forceinline__ MlpView mlp_global(const uint8_t* pk) {
  MlpView v;
  v.w1 = reinterpret_cast<const uint16_t*>(pk + kPkW1);
  v.w2 = reinterpret_cast<const uint16_t*>(pk + kPkW2);
  v.b1 = reinterpret_cast<const float*>(pk + kPkB1);
  v.b2 = reinterpret_cast<const float*>(pk + kPkB2);
  v.w3 = reinterpret_cast<const uint16_t*>(pk + kPkW3);
  v.b3 = *reinterpret_cast<const float*>(pk + kPkB3);
  v.w1s = kMlpInPad;
  v.w2s = kMlpH;
  return v;
}

// LDS copy.  Row strides of 20 and 68 BF16 (40 and 136 bytes) put the 16
// rows one 16-lane group reads at distinct even banks, so the 8-byte A
// operand loads are conflict-free.
constexpr int kW1Ld = 20, kW2Ld = 68, kXsLd = 20;
struct MlpLds {
  uint16_t w1[kMlpH * kW1Ld];
  uint16_t w2[kMlpH * kW2Ld];
  float b1[kMlpH], b2[kMlpH];
  uint16_t w3[kMlpH];
  float b3;
};

// Copies the packed image into L with nthr threads (thread index tid); the
// caller synchronises before use.
__device__ __forceinline__ void mlp_load_lds(MlpLds& L, const uint8_t* __restrict__ pk, int tid,
                                             int nthr) {
  const uint32_t* w1 = reinterpret_cast<const uint32_t*>(pk + kPkW1);
  const uint32_t* w2 = reinterpret_cast<const uint32_t*>(pk + kPkW2);
  for (int i = tid; i < kMlpH * kMlpInPad / 2; i += nthr) {
    const int r = i / (kMlpInPad / 2), k = i % (kMlpInPad / 2);
    reinterpret_cast<uint32_t*>(L.w1)[r * (kW1Ld / 2) + k] = w1[i];
  }
  for (int i = tid; i < kMlpH * kMlpH / 2; i += nthr) {
    const int r = i / (kMlpH / 2), k = i % (kMlpH / 2);
    reinterpret_cast<uint32_t*>(L.w2)[r * (kW2Ld / 2) + k] = w2[i];
  }
  for (int i = tid; i < kMlpH; i += nthr) {
    L.b1[i] = reinterpret_cast<const float*>(pk + kPkB1)[i];
    L.b2[i] = reinterpret_cast<const float*>(pk + kPkB2)[i];
    L.w3[i] = reinterpret_cast<const uint16_t*>(pk + kPkW3)[i];
  }
  if (tid == 0) L.b3 = *reinterpret_cast<const float*>(pk + kPkB3);
}

__device__ __forceinline__ MlpView mlp_lds(const MlpLds& L) {
  MlpView v;
  v.w1 = L.w1;
  v.w2 = L.w2;
  v.b1 = L.b1;
  v.b2 = L.b2;
  v.w3 = L.w3;
  v.b3 = L.b3;
  v.w1s = kW1Ld;
  v.w2s = kW2Ld;
  return v;
}

// Pre-activations of one 16-sample tile t of the staged samples (xs: LDS,
// BF16 rows of stride xss).  a1[mb][r] and a2[mb][r] are hidden unit
// 16 mb + 4 (l/16) + r of sample 16 t + l%16.  Returns that sample's output
// in every lane (after the fold, all four lane groups hold it).  Each stage
// issues all of its operand loads before its first product (scheduling
// barriers keep them there), so their LDS latencies overlap instead of
// adding up one product at a time.
__device__ __forceinline__ float mlp_tile(const MlpView& V, const uint16_t* xs, int xss, int t,
                                          int lane, v4f32* a1, v4f32* a2) {
  const int row = lane & 15, quad = lane >> 4;
  // Layer 1 (K = 16): four independent products.
  const v4s16 xb = load4(xs + (16 * t + row) * xss + 4 * quad);
  v4s16 w1[4];
  v4f32 c1[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const float4 bb = *reinterpret_cast<const float4*>(V.b1 + 16 * mb + 4 * quad);
    c1[mb] = v4f32{bb.x, bb.y, bb.z, bb.w};
    w1[mb] = load4(V.w1 + (16 * mb + row) * V.w1s + 4 * quad);
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) a1[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1[mb], xb, c1[mb], 0, 0, 0);
  uint2 h[4];  // BF16 pairs of the lane's 4 outputs per 16-row block
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    h[mb].x = relu_pk(pk_bf16(a1[mb][0], a1[mb][1]));
    h[mb].y = relu_pk(pk_bf16(a1[mb][2], a1[mb][3]));
  }
  // Layer 2 (K = 64), two 16-unit blocks at a time: two chains of two products.
  const v4u32 b[2] = {{h[0].x, h[0].y, h[1].x, h[1].y}, {h[2].x, h[2].y, h[3].x, h[3].y}};
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    v4u32 w2[2][2];
    v4f32 c2[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int mb = 2 * half + k;
      const float4 bb = *reinterpret_cast<const float4*>(V.b2 + 16 * mb + 4 * quad);
      c2[k] = v4f32{bb.x, bb.y, bb.z, bb.w};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint16_t* wr = V.w2 + (16 * mb + row) * V.w2s + 32 * q + 4 * quad;
        const uint2 lo = *reinterpret_cast<const uint2*>(wr);
        const uint2 hi = *reinterpret_cast<const uint2*>(wr + 16);
        w2[k][q] = v4u32{lo.x, lo.y, hi.x, hi.y};
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int k = 0; k < 2; ++k)
        c2[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16, w2[k][q]),
                                                        __builtin_bit_cast(v8bf16, b[q]), c2[k],
                                                        0, 0, 0);
    a2[2 * half] = c2[0];
    a2[2 * half + 1] = c2[1];
  }
  // Layer 3: every row of A is w3 (same K order as layer 2).
  v4u32 w3[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const uint2 lo = *reinterpret_cast<const uint2*>(V.w3 + 32 * q + 4 * quad);
    const uint2 hi = *reinterpret_cast<const uint2*>(V.w3 + 32 * q + 16 + 4 * quad);
    w3[q] = v4u32{lo.x, lo.y, hi.x, hi.y};
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    h[mb].x = relu_pk(pk_bf16(a2[mb][0], a2[mb][1]));
    h[mb].y = relu_pk(pk_bf16(a2[mb][2], a2[mb][3]));
  }
  v4f32 y = {V.b3, V.b3, V.b3, V.b3};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const v4u32 bq = {h[2 * q].x, h[2 * q].y, h[2 * q + 1].x, h[2 * q + 1].y};
    y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16, w3[q]),
                                                __builtin_bit_cast(v8bf16, bq), y, 0, 0, 0);
  }
  return y[0];
}

// Network outputs of staged rows 0 .. 16 ntiles - 1: lane l receives row
// l's.  All 64 lanes must be active; rows without a sample may hold any
// bits (each output column depends on its own input column only).
__device__ __forceinline__ float mlp_scores(const MlpView& V, const uint16_t* xs, int xss,
                                            int lane, int ntiles) {
  float y = 0.f;
  v4f32 a1[4], a2[4];
#pragma unroll 1
  for (int t = 0; t < ntiles; ++t) {
    // Re-read the weights for every tile (cheap from LDS) instead of letting
    // the compiler keep ~90 VGPRs of them live across the caller's loop.
    asm volatile("" ::: "memory");
    const float s = mlp_tile(V, xs, xss, t, lane, a1, a2);
    if ((lane >> 4) == t) y = s;
  }
  return y;
}

// Stages 12 features as BF16 row `row` (stride xss >= 16, 4 zero columns).
__device__ __forceinline__ void mlp_stage(uint16_t* xs, int xss, int row, const float* f) {
  uint4* r = reinterpret_cast<uint4*>(xs + row * xss);
  r[0] = make_uint4(pk_bf16(f[0], f[1]), pk_bf16(f[2], f[3]), pk_bf16(f[4], f[5]),
                    pk_bf16(f[6], f[7]));
  r[1] = make_uint4(pk_bf16(f[8], f[9]), pk_bf16(f[10], f[11]), 0u, 0u);
}

}  // namespace dev
}  // namespace octgrav
