// Support kernels of the acceptance criteria: FP32 compensated direct
// summation (the accuracy reference of Sec. 3.1, and the learned criterion's
// label normalization), the features + labels of band candidates, and the
// walk records of the centre-of-mass offset opening test.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "octgrav_internal.h"

namespace octgrav {
namespace {

using namespace dev;

constexpr int kThreads = 256;
constexpr int kDTile = 1024;

// Direct sum: one thread per target, all particles streamed through LDS in
// tiles; plain FP32 per tile folded into Neumaier pairs.  The target itself
// contributes -m_i/eps to the potential and nothing to the acceleration;
// that same FP32 value is removed at the end.
__global__ __launch_bounds__(kThreads) void direct_kernel(DevTree T, const int32_t* targets,
                                                          int64_t nt, float eps2, float* acc,
                                                          float* pot) {
  __shared__ float4 src[kDTile];
  const float4* part = reinterpret_cast<const float4*>(T.part);
  const int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool act = u < nt;
  const int64_t i = act ? T.iperm[targets ? targets[u] : u] : 0;
  const float4 xi = part[i];
  Sum4 s;
  s.zero();
  for (int64_t base = 0; base < T.n; base += kDTile) {
    const int cnt = (int)min((int64_t)kDTile, T.n - base);
    for (int k = threadIdx.x; k < cnt; k += kThreads) src[k] = part[base + k];
    __syncthreads();
    if (act) {
      float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
      for (int j = 0; j < cnt; ++j) pp_term(xi, src[j], eps2, ax, ay, az, ph);
      s.fold<false>(ax, ay, az, ph);
    }
    __syncthreads();
  }
  if (act) {
    neu_add(s.s[3], s.c[3], self_term(xi.w, eps2));
    acc[3 * u + 0] = s.s[0] + s.c[0];
    acc[3 * u + 1] = s.s[1] + s.c[1];
    acc[3 * u + 2] = s.s[2] + s.c[2];
    if (pot) pot[u] = s.s[3] + s.c[3];
  }
}

// One block per band pair (group g, cell c): for every target i of g, the
// cell's monopole + quadrupole acceleration against the exact sum over its
// particles, relative to |a_i(direct)|; the label is the largest of them.
// Thread 0 also writes the pair's 12 features.
__global__ __launch_bounds__(kThreads) void mac_label_kernel(DevTree T, WalkBufs B,
                                                             const int32_t* groups, int64_t ngs,
                                                             const int64_t* out_off,
                                                             const float* acc_direct, float eps2,
                                                             float* feat, float* label,
                                                             int32_t* gout, int32_t* cout) {
  __shared__ float red[kThreads * 4];
  __shared__ float emax[kThreads];
  const int64_t p = blockIdx.x;
  // the sampled group this pair belongs to
  int64_t lo = 0, hi = ngs;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (out_off[mid] <= p) lo = mid;
    else hi = mid;
  }
  const int64_t g = groups[lo];
  const int c = B.c_ids[B.c_off[g] + (p - out_off[lo])];
  const int4 gi = reinterpret_cast<const int4*>(T.ginfo)[g];
  const int4 tc = reinterpret_cast<const int4*>(T.topo)[c];
  const float4* part = reinterpret_cast<const float4*>(T.part);
  const float4* mp = reinterpret_cast<const float4*>(T.mp);
  const float4 m0 = mp[3 * (int64_t)c], m1 = mp[3 * (int64_t)c + 1], m2 = mp[3 * (int64_t)c + 2];
  const int tid = threadIdx.x;
  float e_blk = 0.0f;
  for (int off = 0; off < gi.y; off += kChunk) {
    const int nt = min(kChunk, gi.y - off);
    const int S = kThreads / nt, t = tid % nt, slice = tid / nt;
    const float4 xi = part[gi.x + off + t];
    Sum4 s;
    s.zero();
    if (slice < S) {
      float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
      int k = 0;
      for (int j = slice; j < tc.w; j += S) {
        pp_term(xi, part[tc.z + j], eps2, ax, ay, az, ph);
        if (++k == 64) {
          s.fold<false>(ax, ay, az, ph);
          ax = ay = az = ph = 0.f;
          k = 0;
        }
      }
      s.fold<false>(ax, ay, az, ph);
      for (int q = 0; q < 3; ++q) red[4 * tid + q] = s.s[q] + s.c[q];
    }
    __syncthreads();
    if (tid < nt) {
      float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
      for (int sl = 0; sl < S; ++sl) {
        const float* r = red + 4 * (sl * nt + tid);
        neu_add(sx, cx, r[0]);
        neu_add(sy, cy, r[1]);
        neu_add(sz, cz, r[2]);
      }
      float px = 0.f, py = 0.f, pz = 0.f, pp = 0.f;
      pc_term(xi, m0, m1, m2, eps2, px, py, pz, pp);
      const float dx = px - (sx + cx), dy = py - (sy + cy), dz = pz - (sz + cz);
      const int64_t o = T.perm[gi.x + off + tid];
      const float ax = acc_direct[3 * o], ay = acc_direct[3 * o + 1], az = acc_direct[3 * o + 2];
      const float e = sqrtf(dx * dx + dy * dy + dz * dz) / sqrtf(ax * ax + ay * ay + az * az);
      e_blk = fmaxf(e_blk, e);
    }
    __syncthreads();
  }
  emax[tid] = e_blk;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (tid < o) emax[tid] = fmaxf(emax[tid], emax[tid + o]);
    __syncthreads();
  }
  if (tid == 0) {
    label[p] = emax[0];
    const float4* gbox = reinterpret_cast<const float4*>(T.gbox);
    const float4 geo = reinterpret_cast<const float4*>(T.geo)[c];
    const float4* fc = reinterpret_cast<const float4*>(T.fcell);
    if (gout) gout[p] = (int32_t)g;
    if (cout) cout[p] = c;
    mac_features(mac_group(gbox[2 * g], gbox[2 * g + 1]), geo, fc[2 * (int64_t)c],
                 fc[2 * (int64_t)c + 1], feat + 12 * p);
  }
}

// Walk records of the offset opening test at one theta: the boundary of
// each record becomes (com, l + theta |com - cb|) with the leaf sign bit kept,
// the topology is copied, so the walk kernels' own test (d2 == 0 or
// d2 theta^2 < w^2) evaluates the offset criterion unchanged.
__global__ void com_record_kernel(const float4* __restrict__ wrec, const float4* __restrict__ mp,
                                  int64_t nc, float theta, float4* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  const float4 g = wrec[2 * c];
  const float4 m0 = mp[3 * c];
  const float dx = m0.x - g.x, dy = m0.y - g.y, dz = m0.z - g.z;
  const float px = dx * dx, py = dy * dy, pz = dz * dz;
  const float delta = sqrtf((px + py) + pz);  // correctly rounded (HIP default)
  const float td = theta * delta;
  const float lp = fabsf(g.w) + td;
  out[2 * c] = make_float4(m0.x, m0.y, m0.z, copysignf(lp, g.w));
  out[2 * c + 1] = wrec[2 * c + 1];
}

}  // namespace

int launch_com_records(const DevTree& T, float theta, float* out, void* stream) {
  if (T.nc <= 0) return 0;
  com_record_kernel<<<(T.nc + kThreads - 1) / kThreads, kThreads, 0, (hipStream_t)stream>>>(
      reinterpret_cast<const float4*>(T.wrec), reinterpret_cast<const float4*>(T.mp), T.nc, theta,
      reinterpret_cast<float4*>(out));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_direct(const DevTree& T, const int32_t* targets, int64_t nt, float eps, float* acc,
                  float* pot, void* stream) {
  if (nt <= 0) return 0;
  const int64_t grid = (nt + kThreads - 1) / kThreads;
  direct_kernel<<<grid, kThreads, 0, (hipStream_t)stream>>>(T, targets, nt, eps * eps, acc, pot);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mac_labels(const DevTree& T, const WalkBufs& B, const int32_t* groups, int64_t ngs,
                      const int64_t* out_off, const float* acc_direct, float eps, float* feat,
                      float* label, int32_t* gout, int32_t* cout, int64_t npairs, void* stream) {
  if (npairs <= 0) return 0;
  mac_label_kernel<<<npairs, kThreads, 0, (hipStream_t)stream>>>(
      T, B, groups, ngs, out_off, acc_direct, eps * eps, feat, label, gout, cout);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace octgrav
