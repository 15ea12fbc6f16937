// Training and batch inference of the learned acceptance criterion's network
// (12 -> 64 -> 64 -> 1, ReLU; the same network the walk evaluates).
//
// Forward: the wave-level MFMA routine of mlp_device.h over 64 samples per
// wave, keeping the FP32 pre-activations for the backward pass.
// Backward (pinball loss at quantile tau on the log10 error target): one
// thread per sample for the activation gradients, then one thread per
// parameter for the sums over the batch (compensated FP32), with the BF16
// rounding points of the forward pass: weight gradients multiply the rounded
// activation gradients by the rounded activations / inputs; bias gradients
// use the unrounded activation gradients.
// Adam (Kingma & Ba, bias-corrected) on FP32 master weights, after which the
// BF16 inference image is repacked.
#include <hip/hip_runtime.h>

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

// Per sample: loss term, dL/dy, and the activation gradients dh2, dh1
// (unrounded FP32, zero where the unit is inactive).
__global__ __launch_bounds__(256) void mlp_backward_kernel(
    const uint8_t* __restrict__ pk, const float* __restrict__ a1s, const float* __restrict__ a2s,
    const float* __restrict__ y, const float* __restrict__ tgt, int64_t B, float tau,
    float* __restrict__ dh1s, float* __restrict__ dh2s, float* __restrict__ dys,
    float* __restrict__ losss) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const uint16_t* w2 = reinterpret_cast<const uint16_t*>(pk + kPkW2);
  const uint16_t* w3 = reinterpret_cast<const uint16_t*>(pk + kPkW3);
  const float r = tgt[b] - y[b];
  losss[b] = r > 0.f ? tau * r : (tau - 1.f) * r;
  const float dy = (r > 0.f ? -tau : 1.f - tau) / (float)B;
  dys[b] = dy;
  float d2r[kMlpH];
  for (int k = 0; k < kMlpH; ++k) {
    const float d = a2s[b * kMlpH + k] > 0.f ? dy * __uint_as_float((uint32_t)w3[k] << 16) : 0.f;
    dh2s[b * kMlpH + k] = d;
    d2r[k] = bf16_round(d);
  }
  for (int k = 0; k < kMlpH; ++k) {
    float a = 0.f;
    if (a1s[b * kMlpH + k] > 0.f)
      for (int j = 0; j < kMlpH; ++j) a += __uint_as_float((uint32_t)w2[j * kMlpH + k] << 16) * d2r[j];
    dh1s[b * kMlpH + k] = a;
  }
}

__device__ __forceinline__ void kahan(float& s, float& c, float v) {
  const float yv = v - c, t = s + yv;
  c = (t - s) - yv;
  s = t;
}

// Gradient sums over the batch, split over kSplit slices of the batch
// (blockIdx.y): one thread per parameter (plus one for the loss) per slice
// writes a compensated partial sum; mlp_grad_reduce_kernel adds the slices.
constexpr int kSplit = 32;

__global__ __launch_bounds__(256) void mlp_grad_kernel(
    const float* __restrict__ x, const float* __restrict__ a1s, const float* __restrict__ a2s,
    const float* __restrict__ dh1s, const float* __restrict__ dh2s, const float* __restrict__ dys,
    const float* __restrict__ losss, int64_t B, float* __restrict__ part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  const int64_t b0 = B * blockIdx.y / kSplit, b1 = B * (blockIdx.y + 1) / kSplit;
  float s = 0.f, c = 0.f;
  if (p == kMlpParams) {
    for (int64_t b = b0; b < b1; ++b) kahan(s, c, losss[b]);
  } else if (p < kOffB1) {
    const int j = p / kMlpIn, k = p % kMlpIn;
    for (int64_t b = b0; b < b1; ++b)
      kahan(s, c, bf16_round(dh1s[b * kMlpH + j]) * bf16_round(x[b * kMlpIn + k]));
  } else if (p < kOffW2) {
    const int j = p - kOffB1;
    for (int64_t b = b0; b < b1; ++b) kahan(s, c, dh1s[b * kMlpH + j]);
  } else if (p < kOffB2) {
    const int q = p - kOffW2, j = q / kMlpH, k = q % kMlpH;
    for (int64_t b = b0; b < b1; ++b)
      kahan(s, c, bf16_round(dh2s[b * kMlpH + j]) * bf16_round(fmaxf(a1s[b * kMlpH + k], 0.f)));
  } else if (p < kOffW3) {
    const int j = p - kOffB2;
    for (int64_t b = b0; b < b1; ++b) kahan(s, c, dh2s[b * kMlpH + j]);
  } else if (p < kOffB3) {
    const int k = p - kOffW3;
    for (int64_t b = b0; b < b1; ++b) kahan(s, c, dys[b] * bf16_round(fmaxf(a2s[b * kMlpH + k], 0.f)));
  } else {
    for (int64_t b = b0; b < b1; ++b) kahan(s, c, dys[b]);
  }
  part[(int64_t)blockIdx.y * (kMlpParams + 1) + p] = s - c;
}

__global__ __launch_bounds__(256) void mlp_grad_reduce_kernel(const float* __restrict__ part,
                                                              int64_t B, float* __restrict__ grad,
                                                              double* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  if (p == kMlpParams) {
    double s = 0.0;
    for (int k = 0; k < kSplit; ++k) s += (double)part[(int64_t)k * (kMlpParams + 1) + p];
    *loss = s / (double)B;
    return;
  }
  float s = 0.f, c = 0.f;
  for (int k = 0; k < kSplit; ++k) kahan(s, c, part[(int64_t)k * (kMlpParams + 1) + p]);
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

int64_t mlp_grad_scratch_floats() { return (int64_t)kSplit * (kMlpParams + 1); }

int launch_mlp_loss_grad(const void* pk, const float* x, const float* tgt, int64_t B, float tau,
                         float* y, float* a1s, float* a2s, float* dh1s, float* dh2s, float* dys,
                         float* losss, float* part, float* grad, double* loss, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (launch_mlp_forward(pk, x, B, y, a1s, a2s, stream)) return -1;
  mlp_backward_kernel<<<(B + 255) / 256, 256, 0, s>>>((const uint8_t*)pk, a1s, a2s, y, tgt, B, tau,
                                                      dh1s, dh2s, dys, losss);
  const int nb = (kMlpParams + 1 + 255) / 256;
  mlp_grad_kernel<<<dim3(nb, kSplit), 256, 0, s>>>(x, a1s, a2s, dh1s, dh2s, dys, losss, B, part);
  mlp_grad_reduce_kernel<<<nb, 256, 0, s>>>(part, B, grad, loss);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mlp_adam(float* P, float* m, float* v, const float* g, float lr, float b1, float b2,
                    float eps, float c1, float c2, void* stream) {
  mlp_adam_kernel<<<(kMlpParams + 255) / 256, 256, 0, (hipStream_t)stream>>>(P, m, v, g, kMlpParams,
                                                                             lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace octgrav
