// Fused group walk + list evaluation (Sec. 2.2 + 2.3), block-cooperative
// variant for gfx950.
//
// One 256-thread block per work item (a group, or a chunk of 32 of its
// targets) walks the tree breadth-first, 256 candidates per step with an
// order-preserving block-wide compaction, and evaluates accepted cells and
// opened leaves in 256-entry LDS tiles as soon as a tile fills.  Compared with
// the wave-per-item variant it amortizes the walk's per-step work and the
// per-tile work over four waves and larger tiles: the block splits into
// S = floor(256 / n) slices of n lanes, each taking every S-th source of a
// tile.  The lists are identical to the two-pass walk's (same test, same
// breadth-first order); an export mode writes them for the parity tests.
//
// A work item whose frontier outgrows the LDS queue aborts before writing any
// result and is redone by a fallback kernel whose queues live in global
// memory, sized so that they cannot overflow.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "octgrav_internal.h"

namespace octgrav {
namespace {

using namespace dev;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kTile = 256;
constexpr int kRing = 512;  // pending cell ids / leaf ranges (two tiles)

template <int QCAP>
struct BShared {
  int q[QCAP];
  int cring[kRing];
  int2 lring[kRing];  // (first particle, n particles) of opened leaves
  float4 tile[3 * kTile];
  int pre[kTile + 1];
  int lfirst[kTile];
  int wsum[kWaves];
  int wtot[kWaves][3];
};

// Block-wide exclusive scan of one int per thread (wave scans + one exchange).
template <typename SH>
__device__ __forceinline__ int block_excl_scan(int v, SH& sh, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int n = __shfl_up(incl, o);
    if (lane >= o) incl += n;
  }
  if (lane == 63) sh.wsum[wv] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    const int s = sh.wsum[k];
    off += k < wv ? s : 0;
    tot += s;
  }
  *total = tot;
  __syncthreads();
  return off + incl - v;
}

template <bool PLAIN, typename SH>
struct BItem {
  const DevTree& T;
  SH& sh;
  float eps2;
  int tid, nt, S, slice;
  bool active, do_eval;
  float4 xi;
  Sum4 acc4;
  int64_t nsrc = 0;

  __device__ void flush_cells(uint32_t start, int cnt) {
    const float4* mp = reinterpret_cast<const float4*>(T.mp);
    if (do_eval && tid < cnt) {
      const int64_t id = sh.cring[(start + tid) & (kRing - 1)];
      sh.tile[tid] = mp[3 * id];
      sh.tile[kTile + tid] = mp[3 * id + 1];
      sh.tile[2 * kTile + tid] = mp[3 * id + 2];
    }
    __syncthreads();
    if (do_eval && active) {
      float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
      const float4* t0 = sh.tile;
      const float4* t1 = sh.tile + kTile;
      const float4* t2 = sh.tile + 2 * kTile;
      strided2(slice, cnt, S, [&](int j) { pc_term(xi, t0[j], t1[j], t2[j], eps2, ax, ay, az, ph); });
      acc4.template fold<PLAIN>(ax, ay, az, ph);
    }
    __syncthreads();
  }

  __device__ void flush_leaves(uint32_t start, int lc) {
    const float4* part = reinterpret_cast<const float4*>(T.part);
    int ln = 0;
    if (tid < lc) {
      const int2 fl = sh.lring[(start + tid) & (kRing - 1)];
      sh.lfirst[tid] = fl.x;
      ln = fl.y;
    }
    int total;
    const int ex = block_excl_scan(ln, sh, &total);
    if (tid < lc) sh.pre[tid] = ex;
    if (tid == 0) sh.pre[lc] = total;
    nsrc += total;
    __syncthreads();
    if (!do_eval) return;
    for (int u0 = 0; u0 < total; u0 += kTile) {
      const int cnt = min(kTile, total - u0);
      if (tid < cnt) {
        const int u = u0 + tid;
        int lo = 0, hi = lc;  // pre[lo] <= u < pre[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (sh.pre[mid] <= u) lo = mid;
          else hi = mid;
        }
        sh.tile[tid] = part[sh.lfirst[lo] + (u - sh.pre[lo])];
      }
      __syncthreads();
      if (active) {
        float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
        const float4* t0 = sh.tile;
        strided2(slice, cnt, S, [&](int j) { pp_term(xi, t0[j], eps2, ax, ay, az, ph); });
        acc4.template fold<PLAIN>(ax, ay, az, ph);
      }
      __syncthreads();
    }
  }
};

// Walks and evaluates work item w.  Returns false (uniformly, before writing
// any result) if the frontier outgrows the queue.
template <bool PLAIN, typename SH, typename Q>
__device__ bool walk_eval_item(const DevTree& T, const WalkBufs& B, SH& sh, int64_t w,
                               float th2, float eps2, float* __restrict__ acc,
                               float* __restrict__ pot, Q q, uint32_t qmask, bool gmem_q,
                               bool do_eval) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int2 wk = reinterpret_cast<const int2*>(T.work)[w];
  const int64_t g = wk.x;
  const int4 gi = reinterpret_cast<const int4*>(T.ginfo)[g];
  const float4* gbox = reinterpret_cast<const float4*>(T.gbox);
  const float4 gmin = gbox[2 * g], gmax = gbox[2 * g + 1];
  const float4* rec = reinterpret_cast<const float4*>(T.wrec);

  BItem<PLAIN, SH> it{T, sh, eps2};
  it.tid = tid;
  it.nt = min(kChunk, gi.y - wk.y);
  it.S = kThreads / it.nt;
  it.slice = tid / it.nt;
  it.active = it.slice < it.S;
  it.do_eval = do_eval;
  const int first = gi.x + wk.y;
  it.xi = reinterpret_cast<const float4*>(T.part)[first + tid % it.nt];
  it.acc4.zero();

  const bool exp = B.export_lists && wk.y == 0;
  const int64_t xcb = exp ? B.c_off[g] : 0, xce = exp ? B.c_off[g + 1] : 0;
  const int64_t xlb = exp ? B.l_off[g] : 0, xle = exp ? B.l_off[g + 1] : 0;

  uint32_t head = 0, tail = 0, chead = 0, ctail = 0, lhead = 0, ltail = 0;
  const int4 root = reinterpret_cast<const int4*>(rec)[1];
  if (root.y == 0) {  // the root is a leaf: its particles are the whole list
    if (tid == 0) {
      sh.lring[0] = make_int2(root.z, root.w);
      if (exp && xlb < xle) B.l_ids[xlb] = 0;
    }
    ltail = 1;
  } else {
    if (tid < root.y) q[tid] = root.x + tid;
    tail = (uint32_t)root.y;
  }
  if (gmem_q) __threadfence_block();
  __syncthreads();

  while (head < tail) {
    const uint32_t navail = min((uint32_t)kThreads, tail - head);
    const bool valid = (uint32_t)tid < navail;
    int c = 0, nch = 0, kid0 = 0;
    bool toC = false, toL = false;
    int2 leaf_range = make_int2(0, 0);
    uint64_t mC = 0, mL = 0;
    int preN = 0, totN = 0;
    if ((uint32_t)(wv * 64) < navail) {  // this wave has candidates
      float4 ge = make_float4(0.f, 0.f, 0.f, 0.f);
      int4 tp = make_int4(0, 0, 0, 0);
      if (valid) {
        c = (int)q[(head + tid) & qmask];
        ge = rec[2 * (int64_t)c];
        tp = reinterpret_cast<const int4*>(rec)[2 * (int64_t)c + 1];
      }
      const bool op = valid && open_cell(gmin, gmax, ge, th2);
      toC = valid && !op;
      toL = op && tp.y == 0;
      nch = (op && tp.y != 0) ? tp.y : 0;
      kid0 = tp.x;
      leaf_range = make_int2(tp.z, tp.w);
      mC = __ballot(toC);
      mL = __ballot(toL);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint64_t m = __ballot((nch >> b) & 1);
        preN += rank_below(m) << b;
        totN += __popcll(m) << b;
      }
    }
    if (lane == 0) {
      sh.wtot[wv][0] = __popcll(mC);
      sh.wtot[wv][1] = __popcll(mL);
      sh.wtot[wv][2] = totN;
    }
    __syncthreads();
    uint32_t offC = 0, offL = 0, offN = 0, allC = 0, allL = 0, allN = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      const uint32_t a = sh.wtot[k][0], b = sh.wtot[k][1], n = sh.wtot[k][2];
      if (k < wv) {
        offC += a;
        offL += b;
        offN += n;
      }
      allC += a;
      allL += b;
      allN += n;
    }
    if ((tail + allN) - (head + navail) > qmask + 1) return false;
    if (toC) {
      const uint32_t k = ctail + offC + rank_below(mC);
      sh.cring[k & (kRing - 1)] = c;
      if (exp && xcb + k < xce) B.c_ids[xcb + k] = c;
    }
    if (toL) {
      const uint32_t k = ltail + offL + rank_below(mL);
      sh.lring[k & (kRing - 1)] = leaf_range;
      if (exp && xlb + k < xle) B.l_ids[xlb + k] = c;
    }
    const uint32_t base = tail + offN + preN;
    for (int j = 0; j < nch; ++j) q[(base + j) & qmask] = kid0 + j;
    ctail += allC;
    ltail += allL;
    tail += allN;
    head += navail;
    if (gmem_q) __threadfence_block();
    __syncthreads();
    if (ctail - chead >= (uint32_t)kTile) {
      it.flush_cells(chead, kTile);
      chead += kTile;
    }
    if (ltail - lhead >= (uint32_t)kTile) {
      it.flush_leaves(lhead, kTile);
      lhead += kTile;
    }
  }
  while (ctail != chead) {
    const int n = (int)min((uint32_t)kTile, ctail - chead);
    it.flush_cells(chead, n);
    chead += n;
  }
  while (ltail != lhead) {
    const int n = (int)min((uint32_t)kTile, ltail - lhead);
    it.flush_leaves(lhead, n);
    lhead += n;
  }

  if (tid == 0 && wk.y == 0)  // per-group counts; the totals are reduced afterwards
    reinterpret_cast<int4*>(B.cnt)[g] = make_int4((int)ctail, (int)ltail, (int)it.nsrc, 0);
  if (!do_eval) return true;

  // Combine the slices of each target in slice order.
  float* red = reinterpret_cast<float*>(sh.tile);  // [256][8] floats
  if (it.active) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      red[tid * 8 + k] = it.acc4.s[k];
      red[tid * 8 + 4 + k] = it.acc4.c[k];
    }
  }
  __syncthreads();
  if (tid < it.nt) {
    float s[4] = {0.f, 0.f, 0.f, 0.f}, cc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int sl = 0; sl < it.S; ++sl) {
      const float* r = red + (sl * it.nt + tid) * 8;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (PLAIN) {
          s[k] += r[k];
        } else {
          neu_add(s[k], cc[k], r[k]);
          neu_add(s[k], cc[k], r[4 + k]);
        }
      }
    }
    // The target itself is in its own leaf: its self term added -m_i/eps to
    // the potential and nothing to the acceleration; remove that same value.
    const float self = self_term(it.xi.w, eps2);
    if (PLAIN) s[3] += self;
    else neu_add(s[3], cc[3], self);
    const int64_t o = T.perm[first + tid];
    acc[3 * o + 0] = s[0] + cc[0];
    acc[3 * o + 1] = s[1] + cc[1];
    acc[3 * o + 2] = s[2] + cc[2];
    if (pot) pot[o] = s[3] + cc[3];
  }
  __syncthreads();
  return true;
}

template <bool PLAIN, int QCAP>
__global__ __launch_bounds__(kThreads) void walk_eval_block_kernel(DevTree T, WalkBufs B,
                                                                   float th2, float eps2,
                                                                   float* acc, float* pot,
                                                                   int do_eval) {
  __shared__ BShared<QCAP> sh;
  const int64_t w = xcd_slab(blockIdx.x, gridDim.x, T.nw);
  if (w < 0) return;
  const uint32_t qmask = (uint32_t)min(B.lds_qcap, QCAP) - 1;
  if (!walk_eval_item<PLAIN>(T, B, sh, w, th2, eps2, acc, pot, sh.q, qmask, false,
                             do_eval != 0) &&
      threadIdx.x == 0)
    B.ovf_list[atomicAdd(B.ovf_count, 1)] = (int32_t)w;
}

struct GQueue {
  volatile int32_t* p;
  __device__ volatile int32_t& operator[](uint32_t i) const { return p[i]; }
};

template <bool PLAIN>
__global__ __launch_bounds__(kThreads) void walk_eval_block_fallback_kernel(DevTree T, WalkBufs B,
                                                                            float th2, float eps2,
                                                                            float* acc, float* pot,
                                                                            int do_eval) {
  __shared__ BShared<64> sh;
  const int n = *B.ovf_count;
  GQueue q{B.gq + (int64_t)blockIdx.x * B.gq_cap};
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const bool ok = walk_eval_item<PLAIN>(T, B, sh, B.ovf_list[i], th2, eps2, acc, pot, q,
                                          (uint32_t)(B.gq_cap - 1), true, do_eval != 0);
    if (!ok && threadIdx.x == 0) atomicOr(reinterpret_cast<unsigned long long*>(&B.tot[5]), 1ull);
    __syncthreads();
  }
}

__global__ void block_init_kernel(WalkBufs B) {
  if (threadIdx.x < 8) B.tot[threadIdx.x] = 0;
  if (threadIdx.x == 0) *B.ovf_count = 0;
}

}  // namespace

int launch_walk_eval_block(const DevTree& T, const WalkBufs& B, float theta, float eps, bool plain,
                           bool do_eval, float* acc, float* pot, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const float th2 = theta * theta, eps2 = eps * eps;
  const int64_t grid = ((T.nw + 7) / 8) * 8;
  block_init_kernel<<<1, 64, 0, s>>>(B);
  // The breadth-first FIFO holds about two tree levels of the group's walk
  // (peak ~740 entries at theta = 0.5, ~2500 at 0.3 on 2^20 Plummer spheres).
  const bool wide = theta < 0.45f;
  auto go = [&](auto plain_tag) {
    constexpr bool P = decltype(plain_tag)::value;
    if (wide)
      walk_eval_block_kernel<P, 4096><<<grid, kThreads, 0, s>>>(T, B, th2, eps2, acc, pot, do_eval);
    else
      walk_eval_block_kernel<P, 1024><<<grid, kThreads, 0, s>>>(T, B, th2, eps2, acc, pot, do_eval);
    walk_eval_block_fallback_kernel<P><<<B.gq_waves, kThreads, 0, s>>>(T, B, th2, eps2, acc, pot,
                                                                        do_eval);
  };
  if (plain) go(std::true_type{});
  else go(std::false_type{});
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace octgrav
