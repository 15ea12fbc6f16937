// Group tree walk (Sec. 2.2) for gfx950: builds each group's cell list and
// leaf list under the opening angle theta, and the list offsets.
//
// The paper walks with one thread per group and a per-thread stack (the
// tree-walk and test-cell listings).  Here one 64-lane wavefront walks one
// group breadth-first: the frontier is a FIFO of candidate cells in LDS, the
// 64 lanes test 64 candidates at once, and ballots compact the results.
// Because cells are numbered breadth-first with contiguous children, a FIFO
// walk meets candidates in ascending id order, so both lists come out in
// canonical ascending order without a sort.
//
// Two walks as in the paper: a count walk (list sizes), device-side offsets
// (the paper does this prefix sum on the host), then a write walk.  A group
// whose frontier outgrows the LDS queue is flagged by the count walk and
// handled by a fallback walk whose queues live in global memory and are
// sized from the widest tree level, so they cannot overflow.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "octgrav_internal.h"

namespace octgrav {
namespace {

using namespace dev;

constexpr int kFallbackWaves = 2048;

// One wave walks group g.  MODE 0 counts, MODE 1 writes at the offsets,
// MODE 2 counts and writes into the group's fixed-size slots (entries past
// the slot are counted, not written, and flag the call for a redo).
// Q is the frontier storage (LDS, or a volatile global queue in the fallback).
template <int MODE, typename Q>
__device__ void walk_group(const DevTree& T, const WalkBufs& B, int64_t g, float th2, Q q,
                           uint32_t qmask, int fallback) {
  const int lane = threadIdx.x;
  const float4* gbox = reinterpret_cast<const float4*>(T.gbox);
  const float4* rec = reinterpret_cast<const float4*>(T.wrec);
  const float4 gmin = gbox[2 * g], gmax = gbox[2 * g + 1];
  int nC = 0, nL = 0, nsrc = 0, ovf = 0;
  int64_t cb = 0, lb = 0;
  if (MODE == 1) {
    cb = B.c_off[g];
    lb = B.l_off[g];
    if (B.c_off[g + 1] > B.cap_c || B.l_off[g + 1] > B.cap_l) {
      if (lane == 0) atomicOr(reinterpret_cast<unsigned long long*>(&B.tot[4]), 1ull);
      return;
    }
  }
  if (MODE == 2) {
    cb = g * B.slot_c;
    lb = g * B.slot_l;
  }
  const int4 root = reinterpret_cast<const int4*>(rec)[1];
  if (root.y == 0) {  // the root is a leaf: every group sees all particles directly
    if (!B.band) {
      nL = 1;
      nsrc = root.w;
      if (MODE != 0 && lane == 0) B.l_ids[lb] = 0;
    }
  } else {
    uint32_t head = 0, tail = (uint32_t)root.y;
    if (lane < root.y) q[lane] = root.x + lane;
    if (fallback) __threadfence_block();
    __syncthreads();
    while (head < tail) {
      const uint32_t navail = min(64u, tail - head);
      const bool valid = (uint32_t)lane < navail;
      const int c = valid ? (int)q[(head + lane) & qmask] : 0;
      // One 32-byte gather: boundary (test input) and topology (expansion).
      const float4 ge = rec[2 * (int64_t)c];
      const int4 tp = reinterpret_cast<const int4*>(rec)[2 * (int64_t)c + 1];
      const bool op = valid && open_cell(gmin, gmax, ge, th2);
      // Band collection records opened candidates that the wider test at
      // band_hi2 would not open; otherwise the cell / leaf lists of Sec. 2.2.
      const bool toC = B.band ? (op && !open_cell(gmin, gmax, ge, B.band_hi2)) : (valid && !op);
      const bool toL = !B.band && op && tp.y == 0;
      const bool push = op && tp.y != 0;
      const uint64_t mC = __ballot(toC), mL = __ballot(toL);
      if (MODE == 1) {
        if (toC) B.c_ids[cb + nC + rank_below(mC)] = c;
        if (toL) B.l_ids[lb + nL + rank_below(mL)] = c;
      } else {
        if (MODE == 2) {
          const int kc = nC + rank_below(mC), kl = nL + rank_below(mL);
          if (toC && kc < B.slot_c) B.c_ids[cb + kc] = c;
          if (toL && kl < B.slot_l) B.l_ids[lb + kl] = c;
        }
        nsrc += wave_sum(toL ? tp.w : 0);
      }
      nC += __popcll(mC);
      nL += __popcll(mL);
      // Exclusive prefix of the children counts (each <= 8) over the lanes,
      // from one ballot per bit.
      const int nch = push ? tp.y : 0;
      int pre = 0, tot = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint64_t m = __ballot((nch >> b) & 1);
        pre += rank_below(m) << b;
        tot += __popcll(m) << b;
      }
      head += navail;
      if (tail + (uint32_t)tot - head > qmask + 1) {
        ovf = 1;
        break;
      }
      __syncthreads();
      for (int j = 0; j < nch; ++j) q[(tail + pre + j) & qmask] = tp.x + j;
      tail += (uint32_t)tot;
      if (fallback) __threadfence_block();
      __syncthreads();
    }
  }
  if (MODE != 1 && lane == 0) {
    int4 r;
    r.x = nC;
    r.y = nL;
    r.z = nsrc;
    r.w = (ovf || fallback) ? 1 : 0;
    reinterpret_cast<int4*>(B.cnt)[g] = r;
    if (ovf && !fallback) B.ovf_list[atomicAdd(B.ovf_count, 1)] = (int32_t)g;
  }
  if (ovf && fallback && lane == 0)
    atomicOr(reinterpret_cast<unsigned long long*>(&B.tot[5]), 1ull);
}

template <int MODE, int QCAP>
__global__ __launch_bounds__(64) void walk_kernel(DevTree T, WalkBufs B, float th2, int64_t g0,
                                                  int64_t ng) {
  __shared__ int q[QCAP];
  const int64_t i = xcd_slab(blockIdx.x, gridDim.x, ng);
  if (i < 0) return;
  const int64_t g = g0 + i;
  if (MODE == 1 && B.cnt[4 * g + 3]) return;  // walked by the fallback
  walk_group<MODE>(T, B, g, th2, q, (uint32_t)min(B.lds_qcap, QCAP) - 1, 0);
}

// Re-walks the overflowed groups of [g0, g0 + ng) with global-memory queues.
template <int MODE>
__global__ __launch_bounds__(64) void walk_fallback_kernel(DevTree T, WalkBufs B, float th2,
                                                           int64_t g0, int64_t ng) {
  const int n = *B.ovf_count;
  volatile int32_t* q = B.gq + (int64_t)blockIdx.x * B.gq_cap;
  int k = 0;  // index among this range's overflowed groups
  for (int i = 0; i < n; ++i) {
    const int64_t g = B.ovf_list[i];
    if (g < g0 || g >= g0 + ng) continue;
    if (k++ % gridDim.x == blockIdx.x) walk_group<MODE>(T, B, g, th2, q, (uint32_t)(B.gq_cap - 1), 1);
  }
}

__global__ void walk_init_kernel(WalkBufs B) {
  if (threadIdx.x < 8) B.tot[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    *B.ovf_count = 0;
    B.c_off[0] = 0;
    B.l_off[0] = 0;
  }
}

// ----------------------------------------------------------------- offsets
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;

// Exclusive scan of one int64 per thread over a 256-thread block.
__device__ int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    int64_t a = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  int64_t incl = sh[t];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

// Longest cell / leaf list among the groups [a, b) into tot[6] / tot[7]
// (one atomic per block): slot sizes of later slotted calls.
__device__ void block_max_counts(const WalkBufs& B, int64_t a, int64_t b) {
  __shared__ int mx[2];
  if (threadIdx.x == 0) mx[0] = mx[1] = 0;
  __syncthreads();
  int mc = 0, ml = 0;
  for (int64_t g = a + threadIdx.x; g < b; g += blockDim.x) {
    const int4 c = reinterpret_cast<const int4*>(B.cnt)[g];
    mc = max(mc, c.x);
    ml = max(ml, c.y);
  }
  atomicMax(&mx[0], mc);
  atomicMax(&mx[1], ml);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(reinterpret_cast<unsigned long long*>(&B.tot[6]), (unsigned long long)mx[0]);
    atomicMax(reinterpret_cast<unsigned long long*>(&B.tot[7]), (unsigned long long)mx[1]);
  }
  __syncthreads();
}

// Interaction totals of the groups [g0, g0 + ng) from their counts: tot[0..3]
// = cell entries, leaf entries, N_pc, N_pp; tot[6..7] = longest lists;
// tot[4] set if a list outgrew its slot (slot_c > 0).  kTotBlock groups per
// block (a few per thread, so the loads of a thread are few), one pass over
// the counts, one atomic per total and block (integer sums and maxima: the
// result does not depend on the order).
constexpr int kTotBlock = 4 * kScanThreads;
__global__ __launch_bounds__(kScanThreads) void totals_kernel(DevTree T, WalkBufs B, int64_t g0,
                                                              int64_t ng) {
  __shared__ int64_t sh[6][kScanThreads];
  const int64_t a = g0 + (int64_t)blockIdx.x * kTotBlock, b = min(a + kTotBlock, g0 + ng);
  int64_t v[6] = {0, 0, 0, 0, 0, 0};  // sums of 4, maxima of 2
  int ov = 0;
  constexpr int kIt = kTotBlock / kScanThreads;
  int4 cs[kIt];
  int64_t szs[kIt];
#pragma unroll
  for (int it = 0; it < kIt; ++it) {  // every load first (b > a: a clamped index is a group)
    const int64_t g = min(a + threadIdx.x + (int64_t)it * kScanThreads, b - 1);
    cs[it] = reinterpret_cast<const int4*>(B.cnt)[g];
    szs[it] = T.ginfo[4 * g + 1];
  }
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    if (a + threadIdx.x + (int64_t)it * kScanThreads >= b) continue;
    const int4 c = cs[it];
    const int64_t sz = szs[it];
    v[0] += c.x;
    v[1] += c.y;
    v[2] += sz * c.x;
    v[3] += sz * c.z;
    v[4] = max(v[4], (int64_t)c.x);
    v[5] = max(v[5], (int64_t)c.y);
    ov |= B.slot_c > 0 && (c.x > B.slot_c || c.y > B.slot_l);
  }
  for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = v[k];
  const int any_ov = __syncthreads_or(ov);
  for (int o = kScanThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
      for (int k = 4; k < 6; ++k) sh[k][threadIdx.x] = max(sh[k][threadIdx.x], sh[k][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4)
    atomicAdd(reinterpret_cast<unsigned long long*>(&B.tot[threadIdx.x]),
              (unsigned long long)sh[threadIdx.x][0]);
  if (threadIdx.x == 4 || threadIdx.x == 5)
    atomicMax(reinterpret_cast<unsigned long long*>(&B.tot[threadIdx.x + 2]),
              (unsigned long long)sh[threadIdx.x][0]);
  if (threadIdx.x == 0 && any_ov) atomicOr(reinterpret_cast<unsigned long long*>(&B.tot[4]), 1ull);
}

// Offsets of the groups [g0, g0 + ng): per-block sums, then per-block prefix
// of the earlier blocks plus a block scan.  The range's base offset is
// c_off[g0] / l_off[g0] (0 for the first range, else written by the previous
// range's last block), so ranges scanned one after another on one stream
// give the offsets of the whole sequence.
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(DevTree T, WalkBufs B, int64_t g0,
                                                                   int64_t ng) {
  __shared__ int64_t sh[4 * kScanThreads];
  const int64_t base = g0 + (int64_t)blockIdx.x * kScanBlock;
  int64_t sc = 0, sl = 0, npc = 0, npp = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t g = base + threadIdx.x + k * kScanThreads;
    if (g < g0 + ng) {
      const int4 c = reinterpret_cast<const int4*>(B.cnt)[g];
      const int64_t sz = T.ginfo[4 * g + 1];
      sc += c.x;
      sl += c.y;
      npc += sz * c.x;
      npp += sz * c.z;
    }
  }
  block_max_counts(B, base, min(base + kScanBlock, g0 + ng));
  int64_t* s = sh + threadIdx.x;
  s[0] = sc;
  s[kScanThreads] = sl;
  s[2 * kScanThreads] = npc;
  s[3 * kScanThreads] = npp;
  __syncthreads();
  for (int o = kScanThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 4; ++k) s[k * kScanThreads] += s[k * kScanThreads + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    B.blk[2 * blockIdx.x] = sh[0];
    B.blk[2 * blockIdx.x + 1] = sh[kScanThreads];
    atomicAdd(reinterpret_cast<unsigned long long*>(&B.tot[2]), (unsigned long long)sh[2 * kScanThreads]);
    atomicAdd(reinterpret_cast<unsigned long long*>(&B.tot[3]), (unsigned long long)sh[3 * kScanThreads]);
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(DevTree T, WalkBufs B, int64_t g0,
                                                                  int64_t ng) {
  __shared__ int64_t sh[kScanThreads];
  const int64_t c_base = B.c_off[g0], l_base = B.l_off[g0];
  // Offset of this block: the range base plus all earlier blocks' totals.
  int64_t pc = 0, pl = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kScanThreads) {
    pc += B.blk[2 * b];
    pl += B.blk[2 * b + 1];
  }
  int64_t tc, tl;
  block_excl_scan(pc, sh, &tc);
  block_excl_scan(pl, sh, &tl);
  tc += c_base;
  tl += l_base;
  const int64_t base = g0 + (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  int64_t vc[kScanItems], vl[kScanItems], sc = 0, sl = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t g = base + k;
    int4 c = g < g0 + ng ? reinterpret_cast<const int4*>(B.cnt)[g] : make_int4(0, 0, 0, 0);
    vc[k] = c.x;
    vl[k] = c.y;
    sc += c.x;
    sl += c.y;
  }
  int64_t bc, bl;
  int64_t xc = block_excl_scan(sc, sh, &bc) + tc;
  int64_t xl = block_excl_scan(sl, sh, &bl) + tl;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t g = base + k;
    if (g < g0 + ng) {
      B.c_off[g] = xc;
      B.l_off[g] = xl;
    }
    xc += vc[k];
    xl += vl[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
    B.c_off[g0 + ng] = tc + bc;
    B.l_off[g0 + ng] = tl + bl;
    B.tot[0] = tc + bc;
    B.tot[1] = tl + bl;
  }
}

}  // namespace

int64_t scan_scratch_entries(int64_t ng) { return 2 * ((ng + kScanBlock - 1) / kScanBlock + 1); }

int launch_walk(const DevTree& T, const WalkBufs& B, float theta, int mode, void* stream,
                int64_t g0, int64_t ng, bool init) {
  hipStream_t s = (hipStream_t)stream;
  const float th2 = theta * theta;
  if (ng < 0) ng = T.ng - g0;
  const int64_t grid = ((ng + 7) / 8) * 8;
  if (grid == 0) return 0;
  // A wave's breadth-first FIFO holds about two tree levels of its group's
  // walk (peak ~740 entries at theta = 0.5, ~2500 at 0.3 on 2^20 Plummer).
  const bool wide = theta < 0.45f;
  if (mode == 0) {
    if (init) walk_init_kernel<<<1, 64, 0, s>>>(B);
    if (wide) walk_kernel<0, 4096><<<grid, 64, 0, s>>>(T, B, th2, g0, ng);
    else walk_kernel<0, 1024><<<grid, 64, 0, s>>>(T, B, th2, g0, ng);
    walk_fallback_kernel<0><<<B.gq_waves, 64, 0, s>>>(T, B, th2, g0, ng);
  } else if (mode == 2) {
    if (init) walk_init_kernel<<<1, 64, 0, s>>>(B);
    if (wide) walk_kernel<2, 4096><<<grid, 64, 0, s>>>(T, B, th2, g0, ng);
    else walk_kernel<2, 1024><<<grid, 64, 0, s>>>(T, B, th2, g0, ng);
    walk_fallback_kernel<2><<<B.gq_waves, 64, 0, s>>>(T, B, th2, g0, ng);
  } else {
    if (wide) walk_kernel<1, 4096><<<grid, 64, 0, s>>>(T, B, th2, g0, ng);
    else walk_kernel<1, 1024><<<grid, 64, 0, s>>>(T, B, th2, g0, ng);
    walk_fallback_kernel<1><<<B.gq_waves, 64, 0, s>>>(T, B, th2, g0, ng);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_scan(const DevTree& T, const WalkBufs& B, void* stream, int64_t g0, int64_t ng) {
  hipStream_t s = (hipStream_t)stream;
  if (ng < 0) ng = T.ng - g0;
  const int nb = (int)((ng + kScanBlock - 1) / kScanBlock);
  if (nb == 0) return 0;
  scan_reduce_kernel<<<nb, kScanThreads, 0, s>>>(T, B, g0, ng);
  scan_apply_kernel<<<nb, kScanThreads, 0, s>>>(T, B, g0, ng);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_totals(const DevTree& T, const WalkBufs& B, void* stream, int64_t g0, int64_t ng) {
  hipStream_t s = (hipStream_t)stream;
  if (ng < 0) ng = T.ng - g0;
  const int nb = (int)((ng + kTotBlock - 1) / kTotBlock);
  if (nb == 0) return 0;
  totals_kernel<<<nb, kScanThreads, 0, s>>>(T, B, g0, ng);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int fallback_waves() { return kFallbackWaves; }

}  // namespace octgrav
