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

#include <algorithm>
#include <cstdlib>

#include "device_common.h"
#include "octgrav_internal.h"

namespace octgrav {
namespace {

using namespace dev;

constexpr int kThreads = 256;
constexpr int kTile = 256;

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

struct EvalShared {
  float4 buf[3 * kTile];
  int pre[kTile + 1], first[kTile], scan[kThreads];
};

template <bool PLAIN>
__device__ void eval_item(const DevTree& T, const WalkBufs& B, EvalShared& es, float eps2,
                          float* __restrict__ acc, float* __restrict__ pot, int64_t w) {
  float4* shbuf = es.buf;
  float4* sh0 = shbuf;
  float4* sh1 = shbuf + kTile;
  float4* sh2 = shbuf + 2 * kTile;
  int* sh_pre = es.pre;
  int* sh_first = es.first;
  int* sh_scan = es.scan;
  const int tid = threadIdx.x;
  const int2 wk = reinterpret_cast<const int2*>(T.work)[w];
  const int64_t g = wk.x;
  // List ranges: CSR offsets, or per-group slots.  Lists that did not fit
  // are incomplete: skip them, the host redoes the call.
  int64_t c0, c1, l0, l1;
  if (B.slot_c > 0) {
    const int4 cn = reinterpret_cast<const int4*>(B.cnt)[g];
    if (cn.x > B.slot_c || cn.y > B.slot_l) return;  // uniform per block
    c0 = g * B.slot_c;
    c1 = c0 + cn.x;
    l0 = g * B.slot_l;
    l1 = l0 + cn.y;
  } else {
    c0 = B.c_off[g];
    c1 = B.c_off[g + 1];
    l0 = B.l_off[g];
    l1 = B.l_off[g + 1];
    if (c1 > B.cap_c || l1 > B.cap_l) return;  // uniform per block
  }
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
      strided2(slice, cnt, S, [&](int j) { pc_term(xi, sh0[j], sh1[j], sh2[j], eps2, ax, ay, az, ph); });
      acc4.fold<PLAIN>(ax, ay, az, ph);
    }
    __syncthreads();
  }

  // Leaf list: windows of up to 256 leaves; their particles, flattened in
  // list order, are staged in LDS tiles of 256.
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
        strided2(slice, cnt, S, [&](int j) { pp_term(xi, sh0[j], eps2, ax, ay, az, ph); });
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
    const float self = self_term(xi.w, eps2);
    if (PLAIN) s[3] += self;
    else neu_add(s[3], c[3], self);
    const int o = T.perm[first + tid];
    acc[3 * (int64_t)o + 0] = s[0] + c[0];
    acc[3 * (int64_t)o + 1] = s[1] + c[1];
    acc[3 * (int64_t)o + 2] = s[2] + c[2];
    if (pot) pot[o] = s[3] + c[3];
  }
  __syncthreads();
}

// Blocks take the work items [w0, w0 + nw) in XCD slabs; with fewer blocks
// than items each block strides through its slab (grid is a multiple of 8).
template <bool PLAIN>
__global__ __launch_bounds__(kThreads) void eval_kernel(DevTree T, WalkBufs B, float eps2,
                                                        float* __restrict__ acc,
                                                        float* __restrict__ pot, int64_t w0,
                                                        int64_t nw) {
  __shared__ EvalShared es;
  const int64_t nv = ((nw + 7) / 8) * 8;
  for (int64_t v = blockIdx.x; v < nv; v += gridDim.x) {
    const int64_t wi = xcd_slab(v, nv, nw);
    if (wi >= 0) eval_item<PLAIN>(T, B, es, eps2, acc, pot, w0 + wi);
  }
}

// ------------------------------------------------------------ diagnostics
constexpr int kDiagBlocks = 512;

__global__ __launch_bounds__(256) void diag_partial_kernel(DevTree T, const float* acc,
                                                           const float* pot, double* part_sums) {
  __shared__ double sh[4][256];
  double p0 = 0, p1 = 0, p2 = 0, w = 0;
  // In the caller's order: the outputs are read in sequence and only the mass
  // is gathered (through iperm).
  const float4* part = reinterpret_cast<const float4*>(T.part);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < T.n; i += (int64_t)gridDim.x * 256) {
    const double m = part[T.iperm[i]].w;
    p0 += m * (double)acc[3 * i];
    p1 += m * (double)acc[3 * i + 1];
    p2 += m * (double)acc[3 * i + 2];
    if (pot) w += 0.5 * m * (double)pot[i];
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
                float* pot, void* stream, int64_t w0, int64_t nw) {
  hipStream_t s = (hipStream_t)stream;
  const float eps2 = eps * eps;
  if (nw < 0) nw = T.nw - w0;
  const int64_t grid = ((nw + 7) / 8) * 8;
  if (grid == 0) return 0;
  if (plain) eval_kernel<true><<<grid, kThreads, 0, s>>>(T, B, eps2, acc, pot, w0, nw);
  else eval_kernel<false><<<grid, kThreads, 0, s>>>(T, B, eps2, acc, pot, w0, nw);
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
