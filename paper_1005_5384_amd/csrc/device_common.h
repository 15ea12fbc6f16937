// Device helpers shared by the walk and evaluation kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace octgrav {
namespace dev {

// Number of set bits of m below this lane.
__device__ __forceinline__ int rank_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// Wave-uniform copies (scalar registers) of values every lane holds alike:
// per-item constants then stay out of the vector registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)uni((int)(uint32_t)u), hi = (uint32_t)uni((int)(uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float4 uni(float4 v) {
  return make_float4(uni(v.x), uni(v.y), uni(v.z), uni(v.w));
}
__device__ __forceinline__ int4 uni(int4 v) { return make_int4(uni(v.x), uni(v.y), uni(v.z), uni(v.w)); }

__device__ __forceinline__ int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous (Morton-ordered, hence spatially coherent) range of work so that
// neighbouring groups share the XCD's L2.  nblocks is a multiple of 8.
__device__ __forceinline__ int64_t xcd_slab(int64_t b, int64_t nblocks, int64_t n) {
  int64_t per = nblocks >> 3;
  int64_t i = (b & 7) * per + (b >> 3);
  return i < n ? i : -1;
}

// Opening test (Sec. 2.2): open iff d2 == 0 or d2 * theta^2 < l^2, where d is
// the distance from the cell's boundary centre to the group's tight box.
// FP32, this exact operation order, no contraction: the decision is bit-exact
// against any IEEE implementation of the same expression.
__device__ __forceinline__ bool open_cell(float4 gmin, float4 gmax, float4 c, float th2) {
#pragma clang fp contract(off)
  float tx = fmaxf(fmaxf(gmin.x - c.x, c.x - gmax.x), 0.0f);
  float ty = fmaxf(fmaxf(gmin.y - c.y, c.y - gmax.y), 0.0f);
  float tz = fmaxf(fmaxf(gmin.z - c.z, c.z - gmax.z), 0.0f);
  float d2 = (tx * tx + ty * ty) + tz * tz;
  return d2 == 0.0f || d2 * th2 < c.w * c.w;
}

// Particle-particle (body-leaf) term: softened acceleration toward source j
// and potential -m_j / r~, r~^2 = |x_j - x_i|^2 + eps^2.
__device__ __forceinline__ void pp_term(const float4 xi, const float4 sj, float eps2, float& ax,
                                        float& ay, float& az, float& ph) {
  // No contraction: the potential term m_j / r~ is rounded once before it is
  // subtracted, so the self pair's contribution equals self_term() exactly.
#pragma clang fp contract(off)
  const float dx = sj.x - xi.x, dy = sj.y - xi.y, dz = sj.z - xi.z;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
  const float ri = __builtin_amdgcn_rsqf(r2);
  const float mri = sj.w * ri;
  const float mri3 = mri * (ri * ri);
  ax = fmaf(mri3, dx, ax);
  ay = fmaf(mri3, dy, ay);
  az = fmaf(mri3, dz, az);
  ph -= mri;
}

// The self pair's potential term m_i / eps, rounded exactly as pp_term rounds
// it (the walks evaluate the pair j = i and take this value back out).
__device__ __forceinline__ float self_term(float m, float eps2) {
#pragma clang fp contract(off)
  return m * __builtin_amdgcn_rsqf(eps2);
}

// Particle-cell (body-node) term: softened monopole + traceless quadrupole
// about the cell's centre of mass, R = x_i - com, q = Q R, s = R.q:
//   phi += -M/r~ - s/(2 r~^5),  a += -M R/r~^3 + q/r~^5 - 5 s R/(2 r~^7).
// m0 = (com, M), m1 = (Qxx, Qyy, Qzz, Qxy), m2 = (Qxz, Qyz, -, -).
__device__ __forceinline__ void pc_term(const float4 xi, const float4 m0, const float4 m1,
                                        const float4 m2, float eps2, float& ax, float& ay,
                                        float& az, float& ph) {
  const float dx = xi.x - m0.x, dy = xi.y - m0.y, dz = xi.z - m0.z;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
  const float ri = __builtin_amdgcn_rsqf(r2);
  const float ri2 = ri * ri;
  const float qx = fmaf(m2.x, dz, fmaf(m1.w, dy, m1.x * dx));
  const float qy = fmaf(m2.y, dz, fmaf(m1.y, dy, m1.w * dx));
  const float qz = fmaf(m1.z, dz, fmaf(m2.y, dy, m2.x * dx));
  const float s = fmaf(dz, qz, fmaf(dy, qy, dx * qx));
  const float u = s * (ri2 * ri2);
  ph = fmaf(-ri, fmaf(0.5f, u, m0.w), ph);
  const float ri3 = ri * ri2;
  const float c1 = -fmaf(2.5f, u, m0.w) * ri3;
  const float c2 = ri3 * ri2;
  ax = fmaf(c2, qx, fmaf(c1, dx, ax));
  ay = fmaf(c2, qy, fmaf(c1, dy, ay));
  az = fmaf(c2, qz, fmaf(c1, dz, az));
}

// Neumaier compensated addition of v into (s, c).
__device__ __forceinline__ void neu_add(float& s, float& c, float v) {
  const float t = s + v;
  c += (fabsf(s) >= fabsf(v)) ? ((s - t) + v) : ((v - t) + s);
  s = t;
}

// Per-lane accumulator: plain FP32 within a tile, folded per tile into a
// compensated (sum, carry) pair unless PLAIN.
struct Sum4 {
  float s[4], c[4];
  __device__ void zero() {
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] = c[k] = 0.0f;
  }
  template <bool PLAIN>
  __device__ void fold(float a0, float a1, float a2, float a3) {
    if (PLAIN) {
      s[0] += a0;
      s[1] += a1;
      s[2] += a2;
      s[3] += a3;
    } else {
      neu_add(s[0], c[0], a0);
      neu_add(s[1], c[1], a1);
      neu_add(s[2], c[2], a2);
      neu_add(s[3], c[3], a3);
    }
  }
};

// The 12 input features of the learned acceptance criterion for candidate
// cell c seen from a group's tight box, in FP32: f0 = d/l, f1 =
// log10(M/M_tot)/3, f2 = |Q|_F/(M l^2), f3 = log2(1 + r_g/l), f4..6 = cell
// extents / l, f7..9 = log2(1 + group extents / l), f10 = log2(1 +
// depth)/log2(22), f11 = |com - boundary centre| / l.  The cell-only ones
// (f1, f2, f4..6, f10, f11) come precomputed per cell (fc0, fc1); the group's
// part (MacGroup) is computed once per group; f0, f3 and f7..9 use the
// hardware reciprocal, square root and log2 (about 1 ulp each: the features
// are rounded to BF16 for the network).
struct MacGroup {
  float4 gmin, gmax;
  float gx, gy, gz, rg;
};

__device__ __forceinline__ MacGroup mac_group(float4 gmin, float4 gmax) {
#pragma clang fp contract(off)
  MacGroup G;
  G.gmin = gmin;
  G.gmax = gmax;
  G.gx = gmax.x - gmin.x;
  G.gy = gmax.y - gmin.y;
  G.gz = gmax.z - gmin.z;
  G.rg = 0.5f * __builtin_amdgcn_sqrtf((G.gx * G.gx + G.gy * G.gy) + G.gz * G.gz);
  G.gx = uni(G.gx);
  G.gy = uni(G.gy);
  G.gz = uni(G.gz);
  G.rg = uni(G.rg);
  return G;
}

__device__ __forceinline__ void mac_features(const MacGroup& G, float4 geo, float4 fc0,
                                             float4 fc1, float* f) {
#pragma clang fp contract(off)
  const float rl = __builtin_amdgcn_rcpf(fabsf(geo.w));
  const float tx = fmaxf(fmaxf(G.gmin.x - geo.x, geo.x - G.gmax.x), 0.0f);
  const float ty = fmaxf(fmaxf(G.gmin.y - geo.y, geo.y - G.gmax.y), 0.0f);
  const float tz = fmaxf(fmaxf(G.gmin.z - geo.z, geo.z - G.gmax.z), 0.0f);
  f[0] = __builtin_amdgcn_sqrtf((tx * tx + ty * ty) + tz * tz) * rl;
  f[1] = fc0.x;
  f[2] = fc0.y;
  f[3] = __builtin_amdgcn_logf(1.0f + G.rg * rl);
  f[4] = fc0.z;
  f[5] = fc0.w;
  f[6] = fc1.x;
  f[7] = __builtin_amdgcn_logf(1.0f + G.gx * rl);
  f[8] = __builtin_amdgcn_logf(1.0f + G.gy * rl);
  f[9] = __builtin_amdgcn_logf(1.0f + G.gz * rl);
  f[10] = fc1.y;
  f[11] = fc1.z;
}

// Every S-th entry of an LDS tile, starting at `first`, two at a time so the
// compiler can overlap the LDS reads of one term with the arithmetic of the
// other.
template <typename F>
__device__ __forceinline__ void strided2(int first, int cnt, int S, F&& f) {
  int j = first;
  for (; j + S < cnt; j += 2 * S) {
    f(j);
    f(j + S);
  }
  if (j < cnt) f(j);
}

}  // namespace dev
}  // namespace octgrav
