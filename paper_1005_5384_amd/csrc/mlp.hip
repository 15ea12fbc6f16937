// Training and batch inference of the learned acceptance criterion's network
// (12 -> 64 -> 64 -> 1, ReLU; the same network the walk evaluates).
//
// Forward: the wave-level MFMA routine of mlp_device.h over 64 samples per
// wave, keeping the FP32 pre-activations for the backward pass.
// Backward (pinball loss at quantile tau on the log10 error target) on the
// matrix cores as well: dh1 = W2^T d2r per 16-sample tile, then the weight
// gradients as products over slices of the batch, with the BF16 rounding
// points of the forward pass (weight gradients multiply the rounded activation
// gradients by the rounded activations / inputs; bias gradients use the
// unrounded activation gradients); the slices' partial sums are added with
// compensation.
// Adam (Kingma & Ba, bias-corrected) on FP32 master weights, after which the
// BF16 inference image is repacked.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "mlp_device.h"
#include "octgrav_internal.h"

namespace octgrav {
namespace {

using namespace dev;

__global__ void mlp_pack_kernel(const float* __restrict__ P, uint8_t* __restrict__ pk) {
  uint16_t* w1 = reinterpret_cast<uint16_t*>(pk + kPkW1);
  uint16_t* w2 = reinterpret_cast<uint16_t*>(pk + kPkW2);
  float* b1 = reinterpret_cast<float*>(pk + kPkB1);
  float* b2 = reinterpret_cast<float*>(pk + kPkB2);
  uint16_t* w3 = reinterpret_cast<uint16_t*>(pk + kPkW3);
  for (int i = threadIdx.x; i < kMlpH * kMlpInPad; i += blockDim.x) {
    const int j = i / kMlpInPad, k = i % kMlpInPad;
    w1[i] = k < kMlpIn ? (uint16_t)bf16_bits(P[kOffW1 + j * kMlpIn + k]) : (uint16_t)0;
  }
  for (int i = threadIdx.x; i < kMlpH * kMlpH; i += blockDim.x) w2[i] = (uint16_t)bf16_bits(P[kOffW2 + i]);
  for (int i = threadIdx.x; i < kMlpH; i += blockDim.x) {
    b1[i] = P[kOffB1 + i];
    b2[i] = P[kOffB2 + i];
    w3[i] = (uint16_t)bf16_bits(P[kOffW3 + i]);
  }
  if (threadIdx.x == 0) *reinterpret_cast<float*>(pk + kPkB3) = P[kOffB3];
}

// 64 samples per single-wave block; a1s / a2s (B x 64 FP32) may be NULL.
__global__ __launch_bounds__(64) void mlp_forward_kernel(const uint8_t* __restrict__ pk,
                                                         const float* __restrict__ x, int64_t B,
                                                         float* __restrict__ y, float* a1s,
                                                         float* a2s) {
  __shared__ uint16_t xs[64 * kMlpInPad];
  const int lane = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * 64, smp = base + lane;
  float f[kMlpIn];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) f[k] = smp < B ? x[smp * kMlpIn + k] : 0.f;
  mlp_stage(xs, kMlpInPad, lane, f);
  __syncthreads();
  v4f32 a1[4], a2[4];
  const int quad = lane >> 4;
  const MlpView V = mlp_global(pk);
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    const float s = mlp_tile(V, xs, kMlpInPad, t, lane, a1, a2);
    const int64_t st = base + 16 * t + (lane & 15);
    if (st < B && a1s) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        *reinterpret_cast<float4*>(a1s + st * kMlpH + 16 * mb + 4 * quad) =
            make_float4(a1[mb][0], a1[mb][1], a1[mb][2], a1[mb][3]);
        *reinterpret_cast<float4*>(a2s + st * kMlpH + 16 * mb + 4 * quad) =
            make_float4(a2[mb][0], a2[mb][1], a2[mb][2], a2[mb][3]);
      }
    }
    if (quad == t && smp < B) y[smp] = s;
  }
}

// Backward pass of 64 samples per single-wave block, on the matrix cores.
// Per 16-sample tile: the loss terms and dL/dy; dh2 = (a2 > 0) dL/dy w3 and
// its BF16 rounding d2r, built directly in the B-operand layout of the
// 16x16x32 MFMA (lane l: sample l % 16, units 8 (l / 16) .. + 7 of a K step);
// dh1 = (a1 > 0) W2^T d2r as 8 MFMAs (A = rows of W2^T from a transposed LDS
// copy), landing in the D layout (units 4 (l / 16) .. + 3 of each 16-unit
// block).  Written for the gradient sums, unit-major ([unit][sample]) so that
// they are the next products' operands: dh1, dh2 (FP32, for the bias sums)
// and the BF16 roundings of dh1, d2r, relu(a1) and x.
__global__ __launch_bounds__(64) void mlp_backward_kernel(
    const uint8_t* __restrict__ pk, const float* __restrict__ x, const float* __restrict__ a1s,
    const float* __restrict__ a2s, const float* __restrict__ y, const float* __restrict__ tgt,
    int64_t B, float tau, float* __restrict__ dh1T, float* __restrict__ dh2T,
    uint16_t* __restrict__ dh1rT, uint16_t* __restrict__ d2rT, uint16_t* __restrict__ a1rT,
    uint16_t* __restrict__ xrT, float* __restrict__ dys, float* __restrict__ losss) {
  __shared__ __align__(16) uint16_t w2t[kMlpH * kW2Ld];  // W2^T, rows padded like the inference copy
  __shared__ float w3f[kMlpH];
  const int lane = threadIdx.x, row = lane & 15, quad = lane >> 4;
  const uint16_t* w2 = reinterpret_cast<const uint16_t*>(pk + kPkW2);
  for (int i = lane; i < kMlpH * kMlpH; i += 64) {
    const int k = i / kMlpH, j = i % kMlpH;  // W2[k][j]: unit k of layer 2, input j
    w2t[j * kW2Ld + k] = w2[i];
  }
  w3f[lane] = __uint_as_float((uint32_t) reinterpret_cast<const uint16_t*>(pk + kPkW3)[lane] << 16);
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * 64;
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    const int64_t b = base + 16 * t + row;  // this lane's sample
    const bool in = b < B;
    float dy = 0.f;
    if (in) {
      const float r = tgt[b] - y[b];
      dy = (r > 0.f ? -tau : 1.f - tau) / (float)B;
      if (quad == 0) {
        losss[b] = r > 0.f ? tau * r : (tau - 1.f) * r;
        dys[b] = dy;
      }
    }
    // d2r in the B layout, two K steps of 32 units
    v4u32 d2[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k0 = 32 * q + 8 * quad;
      float a[8];
      if (in) {
        const float4 lo = *reinterpret_cast<const float4*>(a2s + b * kMlpH + k0);
        const float4 hi = *reinterpret_cast<const float4*>(a2s + b * kMlpH + k0 + 4);
        a[0] = lo.x; a[1] = lo.y; a[2] = lo.z; a[3] = lo.w;
        a[4] = hi.x; a[5] = hi.y; a[6] = hi.z; a[7] = hi.w;
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = 0.f;
      }
      float d[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        d[i] = a[i] > 0.f ? dy * w3f[k0 + i] : 0.f;
        if (in) {
          dh2T[(int64_t)(k0 + i) * B + b] = d[i];
          d2rT[(int64_t)(k0 + i) * B + b] = (uint16_t)bf16_bits(d[i]);
        }
      }
      d2[q] = v4u32{pk_bf16(d[0], d[1]), pk_bf16(d[2], d[3]), pk_bf16(d[4], d[5]),
                    pk_bf16(d[6], d[7])};
    }
    // dh1 = (a1 > 0) W2^T d2r
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      v4f32 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint16_t* wr = w2t + (16 * mb + row) * kW2Ld + 32 * q + 8 * quad;
        const uint2 lo = *reinterpret_cast<const uint2*>(wr);
        const uint2 hi = *reinterpret_cast<const uint2*>(wr + 4);
        const v4u32 av = {lo.x, lo.y, hi.x, hi.y};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16, av),
                                                    __builtin_bit_cast(v8bf16, d2[q]), c, 0, 0, 0);
      }
      // D layout: units 16 mb + 4 quad + r of sample `row` of this tile
      if (in) {
        const int j0 = 16 * mb + 4 * quad;
        const float4 a1 = *reinterpret_cast<const float4*>(a1s + b * kMlpH + j0);
        const float av[4] = {a1.x, a1.y, a1.z, a1.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float h = av[r] > 0.f ? c[r] : 0.f;
          dh1T[(int64_t)(j0 + r) * B + b] = h;
          dh1rT[(int64_t)(j0 + r) * B + b] = (uint16_t)bf16_bits(h);
          a1rT[(int64_t)(j0 + r) * B + b] = (uint16_t)bf16_bits(fmaxf(av[r], 0.f));
        }
      }
    }
    if (in && quad == 0) {
#pragma unroll
      for (int k = 0; k < kMlpInPad; ++k)
        xrT[(int64_t)k * B + b] = k < kMlpIn ? (uint16_t)bf16_bits(x[b * kMlpIn + k]) : (uint16_t)0;
    }
  }
}

// 8 consecutive BF16 values of row r of a unit-major array (row stride B)
// from sample s on, zero from sample `end` on: one MFMA operand.
__device__ __forceinline__ v4u32 load8(const uint16_t* __restrict__ a, int64_t r, int64_t s,
                                       int64_t B, int64_t end) {
  const uint16_t* p = a + r * B + s;
  if (s + 8 <= end && (((uintptr_t)p) & 3) == 0) {
    const uint2 lo = *reinterpret_cast<const uint2*>(p);
    const uint2 hi = *reinterpret_cast<const uint2*>(p + 4);
    return v4u32{lo.x, lo.y, hi.x, hi.y};
  }
  uint32_t v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t e0 = s + 2 * i < end ? p[2 * i] : 0u;
    const uint32_t e1 = s + 2 * i + 1 < end ? p[2 * i + 1] : 0u;
    v[i] = e0 | (e1 << 16);
  }
  return v4u32{v[0], v[1], v[2], v[3]};
}

// Gradient sums over one slice of the batch (one wave per slice): the weight
// gradients as MFMA products over the slice's samples (the K dimension; exact
// BF16 x BF16 products, FP32 sums), the bias gradients, the w3 gradient and
// the loss on the VALU.  Writes the slice's partial sums; a second kernel adds
// the slices with compensation.
__global__ __launch_bounds__(64) void mlp_grad_kernel(
    const float* __restrict__ a2s, const float* __restrict__ dh1T, const float* __restrict__ dh2T,
    const uint16_t* __restrict__ dh1rT, const uint16_t* __restrict__ d2rT,
    const uint16_t* __restrict__ a1rT, const uint16_t* __restrict__ xrT,
    const float* __restrict__ dys, const float* __restrict__ losss, int64_t B, int64_t slice,
    float* __restrict__ part) {
  const int lane = threadIdx.x, row = lane & 15, quad = lane >> 4;
  const int64_t b0 = (int64_t)blockIdx.x * slice, b1 = min(B, b0 + slice);
  float* out = part + (int64_t)blockIdx.x * (kMlpParams + 1);
  // dW2[k][j] = sum_b d2r[k][b] relu(a1)[j][b]: 4 x 4 output blocks
  v4f32 w2c[4][4];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) w2c[kb][jb] = v4f32{0.f, 0.f, 0.f, 0.f};
  v4f32 w1c[4];
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) w1c[jb] = v4f32{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int64_t s0 = b0; s0 < b1; s0 += 32) {
    const int64_t s = s0 + 8 * quad;
    v4u32 bj[4], ak[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) bj[jb] = load8(a1rT, 16 * jb + row, s, B, b1);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) ak[kb] = load8(d2rT, 16 * kb + row, s, B, b1);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
        w2c[kb][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(v8bf16, ak[kb]), __builtin_bit_cast(v8bf16, bj[jb]), w2c[kb][jb], 0,
            0, 0);
    // dW1[j][i] = sum_b dh1r[j][b] x_r[i][b]
    const v4u32 bx = load8(xrT, row, s, B, b1);
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
      w1c[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          __builtin_bit_cast(v8bf16, load8(dh1rT, 16 * jb + row, s, B, b1)),
          __builtin_bit_cast(v8bf16, bx), w1c[jb], 0, 0, 0);
  }
  // D layout: rows 4 quad + r of each 16-row block, column `row`
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[kOffW2 + (16 * kb + 4 * quad + r) * kMlpH + 16 * jb + row] = w2c[kb][jb][r];
  if (row < kMlpIn) {
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[kOffW1 + (16 * jb + 4 * quad + r) * kMlpIn + row] = w1c[jb][r];
  }
  // biases (unrounded activation gradients), w3 (dL/dy times the rounded
  // relu(a2)), b3 and the loss: lane = unit
  float sb1 = 0.f, sb2 = 0.f, sw3 = 0.f, sb3 = 0.f, sl = 0.f;
  for (int64_t b = b0; b < b1; ++b) {
    sb1 += dh1T[(int64_t)lane * B + b];
    sb2 += dh2T[(int64_t)lane * B + b];
    sw3 += dys[b] * bf16_round(fmaxf(a2s[b * kMlpH + lane], 0.f));
    if (lane == 0) {
      sb3 += dys[b];
      sl += losss[b];
    }
  }
  out[kOffB1 + lane] = sb1;
  out[kOffB2 + lane] = sb2;
  out[kOffW3 + lane] = sw3;
  if (lane == 0) {
    out[kOffB3] = sb3;
    out[kMlpParams] = sl;
  }
}

__device__ __forceinline__ void kahan(float& s, float& c, float v) {
  const float yv = v - c, t = s + yv;
  c = (t - s) - yv;
  s = t;
}

// Sum of the slices' partial sums (compensated), the gradient and the mean
// loss (FP64).
__global__ __launch_bounds__(256) void mlp_grad_reduce_kernel(const float* __restrict__ part,
                                                              int nsl, int64_t B,
                                                              float* __restrict__ grad,
                                                              double* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  if (p == kMlpParams) {
    double s = 0.0;
    for (int k = 0; k < nsl; ++k) s += (double)part[(int64_t)k * (kMlpParams + 1) + p];
    *loss = s / (double)B;
    return;
  }
  float s = 0.f, c = 0.f;
  for (int k = 0; k < nsl; ++k) kahan(s, c, part[(int64_t)k * (kMlpParams + 1) + p]);
  grad[p] = s - c;
}

__global__ void mlp_adam_kernel(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                                const float* __restrict__ g, int n, float lr, float b1, float b2,
                                float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

int launch_mlp_pack(const float* P, void* pk, void* stream) {
  mlp_pack_kernel<<<1, 256, 0, (hipStream_t)stream>>>(P, (uint8_t*)pk);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mlp_forward(const void* pk, const float* x, int64_t B, float* y, float* a1s, float* a2s,
                       void* stream) {
  if (B <= 0) return 0;
  mlp_forward_kernel<<<(B + 63) / 64, 64, 0, (hipStream_t)stream>>>((const uint8_t*)pk, x, B, y,
                                                                   a1s, a2s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Batch slices of the gradient sums: at most kMaxSlices, whole K steps of 32.
constexpr int64_t kMaxSlices = 256;
static int64_t slice_len(int64_t B) {
  const int64_t nsl = std::min<int64_t>(kMaxSlices, (B + 63) / 64);
  return ((B + nsl - 1) / nsl + 31) / 32 * 32;
}

int64_t mlp_train_scratch_floats(int64_t B) {
  // y, dL/dy, loss terms; a1, a2, dh1^T, dh2^T (FP32); dh1r^T, d2r^T, relu(a1)r^T
  // (BF16, 64 rows) and x_r^T (BF16, 16 rows); the slices' partial sums
  return 3 * B + 4 * kMlpH * B + (3 * kMlpH + kMlpInPad) * B / 2 + 4 + kMaxSlices * (kMlpParams + 1);
}

int launch_mlp_loss_grad(const void* pk, const float* x, const float* tgt, int64_t B, float tau,
                         float* scratch, float* grad, double* loss, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  float *y = scratch, *dys = y + B, *losss = dys + B, *a1 = losss + B, *a2 = a1 + kMlpH * B,
        *dh1T = a2 + kMlpH * B, *dh2T = dh1T + kMlpH * B;
  uint16_t* dh1rT = reinterpret_cast<uint16_t*>(dh2T + kMlpH * B);
  uint16_t *d2rT = dh1rT + kMlpH * B, *a1rT = d2rT + kMlpH * B, *xrT = a1rT + kMlpH * B;
  float* part = reinterpret_cast<float*>(
      (reinterpret_cast<uintptr_t>(xrT + kMlpInPad * B) + 15) & ~uintptr_t(15));  // <= 4 floats on
  if (launch_mlp_forward(pk, x, B, y, a1, a2, stream)) return -1;
  mlp_backward_kernel<<<(B + 63) / 64, 64, 0, s>>>((const uint8_t*)pk, x, a1, a2, y, tgt, B, tau,
                                                   dh1T, dh2T, dh1rT, d2rT, a1rT, xrT, dys, losss);
  const int64_t sl = slice_len(B);
  const int nsl = (int)((B + sl - 1) / sl);
  mlp_grad_kernel<<<nsl, 64, 0, s>>>(a2, dh1T, dh2T, dh1rT, d2rT, a1rT, xrT, dys, losss, B, sl,
                                     part);
  mlp_grad_reduce_kernel<<<(kMlpParams + 1 + 255) / 256, 256, 0, s>>>(part, nsl, B, grad, loss);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mlp_adam(float* P, float* m, float* v, const float* g, float lr, float b1, float b2,
                    float eps, float c1, float c2, void* stream) {
  mlp_adam_kernel<<<(kMlpParams + 255) / 256, 256, 0, (hipStream_t)stream>>>(P, m, v, g, kMlpParams,
                                                                             lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace octgrav
