// Evaluation of the interaction lists (Sec. 2.3) for gfx950, plus the FP64
// momentum/energy diagnostics.
//
// The paper gives each group a block with one thread per particle and
// streams block-size tiles of cells (the body-node listing) and of leaf
// particles (the body-leaf listing) through shared memory.  Its groups hold
// a third to a quarter of N_group particles on average, so most threads
// idle.  Here a 256-thread block takes one work item (a group, or a chunk of
// 64 of its targets) and splits itself into S = floor(256 / n) slices of n
// lanes: every slice holds all n targets and takes every S-th source of each
// LDS tile, and the slices' partial sums are combined at the end in a fixed
// order.  Sources are broadcast from LDS (all lanes of a slice read the same
// entry).  Arithmetic is FP32 with v_rsq_f32; each lane accumulates a tile
// in plain FP32 and folds it into a Neumaier-compensated (sum, carry) pair.
#include <hip/hip_runtime.h>

#include "octgrav_internal.h"

namespace octgrav {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 256;

__device__ __forceinline__ int64_t xcd_slab(int64_t b, int64_t nblocks, int64_t n) {
  int64_t per = nblocks >> 3;
  int64_t i = (b & 7) * per + (b >> 3);
  return i < n ? i : -1;
}

// Particle-particle (body-leaf) term: softened acceleration toward source j
// and potential -m_j / r~, r~^2 = |x_j - x_i|^2 + eps^2.
__device__ __forceinline__ void pp_term(const float4 xi, const float4 sj, float eps2, float& ax,
                                        float& ay, float& az, float& ph) {
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

// Block-wide exclusive scan of one int per thread (256 threads).
__device__ int block_excl_scan_int(int v, int* sh, int* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kThreads; o <<= 1) {
    int a = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const int incl = sh[t];
  *total = sh[kThreads - 1];
  __syncthreads();
  return incl - v;
}

template <bool PLAIN>
__global__ __launch_bounds__(kThreads) void eval_kernel(DevTree T, WalkBufs B, float eps2,
                                                        float* __restrict__ acc,
                                                        float* __restrict__ pot) {
  __shared__ float4 shbuf[3 * kTile];
  float4* sh0 = shbuf;
  float4* sh1 = shbuf + kTile;
  float4* sh2 = shbuf + 2 * kTile;
  __shared__ int sh_pre[kTile + 1], sh_first[kTile], sh_scan[kThreads];
  const int64_t w = xcd_slab(blockIdx.x, gridDim.x, T.nw);
  if (w < 0) return;
  if (B.tot[0] > B.cap_c || B.tot[1] > B.cap_l) return;  // lists incomplete: the host retries
  const int tid = threadIdx.x;
  const int2 wk = reinterpret_cast<const int2*>(T.work)[w];
  const int64_t g = wk.x;
  const int4 gi = reinterpret_cast<const int4*>(T.ginfo)[g];
  const int first = gi.x + wk.y;
  const int nt = min(kChunk, gi.y - wk.y);
  const int S = kThreads / nt;
  const int t = tid % nt, slice = tid / nt;
  const bool active = slice < S;
  const float4* part = reinterpret_cast<const float4*>(T.part);
  const float4* mp = reinterpret_cast<const float4*>(T.mp);
  const int4* topo = reinterpret_cast<const int4*>(T.topo);
  const float4 xi = part[first + t];
  Sum4 acc4;
  acc4.zero();

  // Cell list: tiles of up to 256 cells' moments staged in LDS.
  const int64_t c0 = B.c_off[g], c1 = B.c_off[g + 1];
  for (int64_t base = c0; base < c1; base += kTile) {
    const int cnt = (int)min((int64_t)kTile, c1 - base);
    if (tid < cnt) {
      const int id = B.c_ids[base + tid];
      sh0[tid] = mp[3 * (int64_t)id];
      sh1[tid] = mp[3 * (int64_t)id + 1];
      sh2[tid] = mp[3 * (int64_t)id + 2];
    }
    __syncthreads();
    if (active) {
      float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
      for (int j = slice; j < cnt; j += S) pc_term(xi, sh0[j], sh1[j], sh2[j], eps2, ax, ay, az, ph);
      acc4.fold<PLAIN>(ax, ay, az, ph);
    }
    __syncthreads();
  }

  // Leaf list: windows of up to 256 leaves; their particles, flattened in
  // list order, are staged in LDS tiles of 256.
  const int64_t l0 = B.l_off[g], l1 = B.l_off[g + 1];
  for (int64_t lb = l0; lb < l1; lb += kTile) {
    const int lc = (int)min((int64_t)kTile, l1 - lb);
    int ln = 0;
    if (tid < lc) {
      const int4 tp = topo[B.l_ids[lb + tid]];
      sh_first[tid] = tp.z;
      ln = tp.w;
    }
    int total;
    const int ex = block_excl_scan_int(ln, sh_scan, &total);
    if (tid < lc) sh_pre[tid] = ex;
    if (tid == 0) sh_pre[lc] = total;
    __syncthreads();
    for (int u0 = 0; u0 < total; u0 += kTile) {
      const int cnt = min(kTile, total - u0);
      if (tid < cnt) {
        const int u = u0 + tid;
        int lo = 0, hi = lc;  // sh_pre[lo] <= u < sh_pre[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (sh_pre[mid] <= u) lo = mid;
          else hi = mid;
        }
        sh0[tid] = part[sh_first[lo] + (u - sh_pre[lo])];
      }
      __syncthreads();
      if (active) {
        float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
        for (int j = slice; j < cnt; j += S) pp_term(xi, sh0[j], eps2, ax, ay, az, ph);
        acc4.fold<PLAIN>(ax, ay, az, ph);
      }
      __syncthreads();
    }
  }

  // Combine the slices of each target in slice order.
  float* red = reinterpret_cast<float*>(shbuf);  // [256][8] floats
  if (active) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      red[tid * 8 + k] = acc4.s[k];
      red[tid * 8 + 4 + k] = acc4.c[k];
    }
  }
  __syncthreads();
  if (tid < nt) {
    float s[4] = {0.f, 0.f, 0.f, 0.f}, c[4] = {0.f, 0.f, 0.f, 0.f};
    for (int sl = 0; sl < S; ++sl) {
      const float* r = red + (sl * nt + tid) * 8;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (PLAIN) {
          s[k] += r[k];
        } else {
          neu_add(s[k], c[k], r[k]);
          neu_add(s[k], c[k], r[4 + k]);
        }
      }
    }
    // The leaf list holds the target itself; its self term contributed
    // -m_i/eps to the potential and nothing to the acceleration.  Remove it
    // with the identical FP32 value.
    const float self = xi.w * __builtin_amdgcn_rsqf(eps2);
    if (PLAIN) s[3] += self;
    else neu_add(s[3], c[3], self);
    const int o = T.perm[first + tid];
    acc[3 * (int64_t)o + 0] = s[0] + c[0];
    acc[3 * (int64_t)o + 1] = s[1] + c[1];
    acc[3 * (int64_t)o + 2] = s[2] + c[2];
    if (pot) pot[o] = s[3] + c[3];
  }
}

// ------------------------------------------------------------ diagnostics
constexpr int kDiagBlocks = 512;

__global__ __launch_bounds__(256) void diag_partial_kernel(DevTree T, const float* acc,
                                                           const float* pot, double* part_sums) {
  __shared__ double sh[4][256];
  double p0 = 0, p1 = 0, p2 = 0, w = 0;
  const float4* part = reinterpret_cast<const float4*>(T.part);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < T.n; i += (int64_t)gridDim.x * 256) {
    const double m = part[i].w;
    const int64_t o = T.perm[i];
    p0 += m * (double)acc[3 * o];
    p1 += m * (double)acc[3 * o + 1];
    p2 += m * (double)acc[3 * o + 2];
    if (pot) w += 0.5 * m * (double)pot[o];
  }
  sh[0][threadIdx.x] = p0;
  sh[1][threadIdx.x] = p1;
  sh[2][threadIdx.x] = p2;
  sh[3][threadIdx.x] = w;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 4) part_sums[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void diag_final_kernel(const double* part_sums, int nb,
                                                         double* out4) {
  __shared__ double sh[4][256];
  double v[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += 256)
    for (int k = 0; k < 4; ++k) v[k] += part_sums[4 * b + k];
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 4) out4[threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace

int launch_eval(const DevTree& T, const WalkBufs& B, float eps, bool plain, float* acc,
                float* pot, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const float eps2 = eps * eps;
  const int64_t grid = ((T.nw + 7) / 8) * 8;
  if (plain) eval_kernel<true><<<grid, kThreads, 0, s>>>(T, B, eps2, acc, pot);
  else eval_kernel<false><<<grid, kThreads, 0, s>>>(T, B, eps2, acc, pot);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int64_t diag_scratch_entries(int64_t) { return 4 * kDiagBlocks; }

int launch_diag(const DevTree& T, const float* acc, const float* pot, double* part_sums,
                double* out4, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  diag_partial_kernel<<<kDiagBlocks, 256, 0, s>>>(T, acc, pot, part_sums);
  diag_final_kernel<<<1, 256, 0, s>>>(part_sums, kDiagBlocks, out4);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace octgrav
