// Octree construction on the GPU (the host build of Sec. 2.1 moved to the
// device), bit-identical to the host build: the same 63-bit Morton keys from
// the same FP64 grid arithmetic, a stable radix sort (ties by input index),
// the same level-synchronous breadth-first subdivision, and FP64 boxes and
// moments bottom-up with the host's operation order (no contraction, the
// host's min / max), so every exported array matches bitwise.
//
// Per level: one thread per cell finds its octant boundaries by binary search
// in the sorted keys and counts non-empty children; a scan numbers the
// children; a second pass writes them.  Boxes and moments: one thread per
// cell, deepest level first.  Then the FP32 images, the walk records, the
// learned criterion's cell features, the groups (scattered to their first
// particle and compacted, which orders them by first particle) and the work
// chunks.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstring>
#include <vector>

#include "octgrav_internal.h"

namespace octgrav {
namespace {

constexpr uint32_t kGridMax = (1u << kMaxDepth) - 1;
constexpr int kT = 256;

inline int blocks(int64_t n) { return (int)((n + kT - 1) / kT); }

// Bounding box: per-block min / max of each coordinate (FP32 values are
// exact in FP64, so the order of the reduction does not matter).
// With mass != nullptr (inputs already on the device) it also checks them in
// the same pass: bit 1 of *bad = a position not finite or |x| >= 2^60, bit 2
// = a mass not finite or not > 0.
__global__ void bbox_kernel(const float* __restrict__ pos, const float* __restrict__ mass,
                            int64_t n, float* __restrict__ part, int32_t* __restrict__ bad) {
  __shared__ float sh[6][kT];
  // min / max with the host's tie rule (keeps the earlier of equal values,
  // so +0 / -0 resolve as they do on the host)
  float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  int bd = 0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    for (int k = 0; k < 3; ++k) {
      const float x = pos[3 * i + k];
      v[k] = x < v[k] ? x : v[k];
      v[3 + k] = v[3 + k] < x ? x : v[3 + k];
      if (!(fabsf(x) < 0x1p60f)) bd |= 1;  // also catches NaN
    }
    if (mass) {
      const float m = mass[i];
      if (!(m > 0.0f) || !(m < INFINITY)) bd |= 2;
    }
  }
  if (mass) {
    if (__any(bd & 1) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
    if (__any(bd & 2) && (threadIdx.x & 63) == 0) atomicOr(bad, 2);
  }
  for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 6; ++k) {
        const float a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + o];
        sh[k][threadIdx.x] = k < 3 ? (b < a ? b : a) : (a < b ? b : a);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// Root cube from the bounding-box partials with the host's rules (min / max
// keeping the earlier of equal values, combined over contiguous ranges in
// index order; the cube of the largest extent rounded up to a power of two,
// centred on the box; FP64, the same operations): cube = corner xyz, side,
// grid step, 1 / step.  One block of kT threads.
__global__ __launch_bounds__(kT) void root_kernel(const float* __restrict__ part, int nbb,
                                                  double* __restrict__ cube) {
#pragma clang fp contract(off)
  __shared__ float sh[6][kT];
  const int t = threadIdx.x, per = (nbb + kT - 1) / kT;
  float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int i = t * per; i < min(nbb, (t + 1) * per); ++i)
    for (int k = 0; k < 3; ++k) {
      const float x = part[6 * i + k], y = part[6 * i + 3 + k];
      v[k] = x < v[k] ? x : v[k];
      v[3 + k] = v[3 + k] < y ? y : v[3 + k];
    }
  for (int k = 0; k < 6; ++k) sh[k][t] = v[k];
  __syncthreads();
  for (int w = 1; w < kT; w <<= 1) {  // thread t holds [t, t + 2w) after this step
    if ((t & (2 * w - 1)) == 0)
      for (int k = 0; k < 6; ++k) {
        const float a = sh[k][t], b = sh[k][t + w];
        sh[k][t] = k < 3 ? (b < a ? b : a) : (a < b ? b : a);
      }
    __syncthreads();
  }
  if (t != 0) return;
  double lo[3], hi[3];
  for (int k = 0; k < 3; ++k) {
    lo[k] = sh[k][0];
    hi[k] = sh[3 + k][0];
  }
  const double e1 = hi[1] - lo[1], e2 = hi[2] - lo[2], e0 = hi[0] - lo[0];
  const double e12 = e1 < e2 ? e2 : e1;
  const double ext = e0 < e12 ? e12 : e0;
  int e = 1;
  if (ext > 0) (void)frexp(ext, &e);
  const double side = ext > 0 ? ldexp(1.0, e) : 1.0;
  for (int k = 0; k < 3; ++k) cube[k] = (lo[k] + hi[k]) * 0.5 - 0.5 * side;
  cube[3] = side;
  cube[4] = ldexp(side, -kMaxDepth);
  cube[5] = ldexp(1.0 / side, kMaxDepth);
}

// The host's grid coordinate: floor, then exact against the grid planes.
__device__ __forceinline__ uint32_t grid_coord(double x, double corner, double step,
                                               double inv_step) {
#pragma clang fp contract(off)
  const double f = floor((x - corner) * inv_step);
  int64_t u = f < 0 ? 0 : (f > (double)kGridMax ? (int64_t)kGridMax : (int64_t)f);
  while (u > 0 && corner + (double)u * step > x) --u;
  while (u < (int64_t)kGridMax && corner + (double)(u + 1) * step <= x) ++u;
  return (uint32_t)u;
}

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

// cube: corner xyz, side, grid step, 1 / step (root_kernel).  Also packs
// each particle as (x, y, z, m) in input order, so that the gather after the
// sort reads one aligned 16-byte record per particle.
__global__ void keys_kernel(const float* __restrict__ pos, const float* __restrict__ mass,
                            int64_t n, const double* __restrict__ cube,
                            uint64_t* __restrict__ key, int32_t* __restrict__ idx,
                            float4* __restrict__ packed) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const double step = cube[4], inv = cube[5];
  const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  const uint32_t u0 = grid_coord((double)x, cube[0], step, inv);
  const uint32_t u1 = grid_coord((double)y, cube[1], step, inv);
  const uint32_t u2 = grid_coord((double)z, cube[2], step, inv);
  key[i] = spread3(u0) | spread3(u1) << 1 | spread3(u2) << 2;
  idx[i] = (int32_t)i;
  packed[i] = make_float4(x, y, z, mass[i]);
}

struct Cells {
  int32_t* first;   // first particle
  int32_t* n;       // particles
  int32_t* depth;
  int32_t* parent;
  int32_t* fc;      // first child (-1)
  int32_t* nc;      // children
};

// Octant boundaries of the level's cells [lbeg, lbeg + m) at digit shift sh;
// bd[9 j ..] and the count of non-empty children of cell lbeg + j.
__global__ void split_kernel(Cells C, const uint64_t* __restrict__ key, int64_t lbeg, int64_t m,
                             int L, int n_leaf, int32_t* __restrict__ bd,
                             int32_t* __restrict__ nkid) {
  const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (j >= m) return;
  const int64_t c = lbeg + j;
  const int32_t a = C.first[c], b = a + C.n[c];
  if (C.n[c] <= n_leaf || L == kMaxDepth) {
    nkid[j] = 0;
    return;
  }
  const int sh = 3 * (kMaxDepth - 1 - L);
  int32_t* d9 = bd + 9 * j;
  d9[0] = a;
  int32_t lo = a;
  int cnt = 0;
  for (int d = 1; d < 8; ++d) {
    // first index in [lo, b) whose digit is >= d (digits are sorted)
    int32_t l = lo, h = b;
    while (l < h) {
      const int32_t mid = l + ((h - l) >> 1);
      if ((int)((key[mid] >> sh) & 7) < d) l = mid + 1;
      else h = mid;
    }
    d9[d] = l;
    cnt += l > lo;
    lo = l;
  }
  d9[8] = b;
  cnt += b > lo;
  nkid[j] = cnt;
}

__global__ void emit_kernel(Cells C, int64_t lbeg, int64_t lend, int64_t m, int L,
                            const int32_t* __restrict__ bd, const int32_t* __restrict__ nkid,
                            const int32_t* __restrict__ pre) {
  const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (j >= m || nkid[j] == 0) return;
  const int64_t c = lbeg + j;
  int64_t ch = lend + pre[j];
  C.fc[c] = (int32_t)ch;
  C.nc[c] = nkid[j];
  const int32_t* d9 = bd + 9 * j;
  for (int d = 0; d < 8; ++d)
    if (d9[d + 1] > d9[d]) {
      C.first[ch] = d9[d];
      C.n[ch] = d9[d + 1] - d9[d];
      C.depth[ch] = L + 1;
      C.parent[ch] = (int32_t)c;
      C.fc[ch] = -1;
      C.nc[ch] = 0;
      ++ch;
    }
}

// ---- subdivision without host round trips: every level's range lives on
// the device, so all levels are launched back to back.
struct Level {
  int64_t beg, end;   // the level's cells [beg, end)
  int64_t total;      // children it emitted
  int32_t overflow;   // the cell arrays could not hold them
  int32_t pad;
};
constexpr int kLB = 512;  // blocks of the level kernels; block b owns a contiguous chunk

// Eight lanes per cell: lane d of the group finds the first particle of the
// cell whose octant digit at level L is >= d (d = 0: the cell's first), all
// eight searches at once; the next lane's boundary closes the octant.
// Returns whether octant d is a non-empty child (false for leaves).
struct OctantLane {
  int64_t c;
  int32_t lo, hi;  // the octant's particles [lo, hi)
  bool child;
};
__device__ OctantLane octant_lane(const Cells& C, const uint64_t* __restrict__ key, int64_t beg,
                                  int64_t j, bool valid, int L, int n_leaf) {
  const int d = threadIdx.x & 7;
  OctantLane o{beg + j, 0, 0, false};
  int32_t a = 0, b = 0;
  bool split = false;
  if (valid) {
    a = C.first[o.c];
    b = a + C.n[o.c];
    split = !(C.n[o.c] <= n_leaf || L == kMaxDepth);
  }
  int32_t l = a;
  if (split && d > 0) {
    const int sh = 3 * (kMaxDepth - 1 - L);
    int32_t h = b;
    while (l < h) {
      const int32_t mid = l + ((h - l) >> 1);
      if ((int)((key[mid] >> sh) & 7) < d) l = mid + 1;
      else h = mid;
    }
  }
  const int32_t nx = __shfl_down(l, 1, 8);
  o.lo = l;
  o.hi = d == 7 ? b : nx;
  o.child = split && o.hi > o.lo;
  return o;
}

// octant_lane from the boundaries split_level_kernel stored (bnd[8 j + d] =
// lane d's search result, the cell's first particle where nothing was
// searched): the same result without the searches.
__device__ OctantLane octant_lane_stored(const Cells& C, const int32_t* __restrict__ bnd,
                                         int64_t beg, int64_t j, bool valid, int L, int n_leaf) {
  const int d = threadIdx.x & 7;
  OctantLane o{beg + j, 0, 0, false};
  int32_t b = 0, l = 0;
  bool split = false;
  if (valid) {
    b = C.first[o.c] + C.n[o.c];
    split = !(C.n[o.c] <= n_leaf || L == kMaxDepth);
    l = bnd[8 * j + d];
  }
  const int32_t nx = __shfl_down(l, 1, 8);
  o.lo = l;
  o.hi = d == 7 ? b : nx;
  o.child = split && o.hi > o.lo;
  return o;
}

// Non-empty children among the eight lanes of this lane's group, and how many
// of them come before this lane.
__device__ void octant_counts(bool child, int* n, int* before) {
  const uint64_t m = __ballot(child);
  const int lane = threadIdx.x & 63, g = lane & ~7;
  const uint32_t grp = (uint32_t)(m >> g) & 0xffu;
  *n = __popc(grp);
  *before = __popc(grp & ((1u << (lane - g)) - 1u));
}

// Sum of v over the block (kT threads); every thread gets it.
__device__ int block_sum(int v, int* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
  for (int k = 0; k < kT / 64; ++k) t += sh[k];
  __syncthreads();
  return t;
}

// Exclusive prefix of v over the block in thread order, and the block total.
__device__ int block_exclusive(int v, int* total, int* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  int base = 0, tot = 0;
  for (int k = 0; k < kT / 64; ++k) {
    base += k < w ? sh[k] : 0;
    tot += sh[k];
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

__global__ void level_init_kernel(Cells C, Level* lv, int32_t n) {
  if (threadIdx.x == 0) {
    C.first[0] = 0;
    C.n[0] = n;
    C.depth[0] = 0;
    C.parent[0] = -1;
    C.fc[0] = -1;
    C.nc[0] = 0;
  }
  if (threadIdx.x < kMaxDepth + 2) {
    const int64_t e = threadIdx.x == 0 ? 1 : 0;
    lv[threadIdx.x] = Level{0, e, 0, 0, 0};
  }
}

// Children of level L's cells counted per block (bsum); eight lanes per
// cell.  A level of at most bcap cells also keeps the octant boundaries in
// bnd for emit_level_kernel.
__global__ __launch_bounds__(kT) void split_level_kernel(Cells C, const uint64_t* __restrict__ key,
                                                         const Level* __restrict__ lv, int L,
                                                         int n_leaf, int32_t* __restrict__ bsum,
                                                         int32_t* __restrict__ bnd, int64_t bcap) {
  __shared__ int sh[kT / 64];
  const int64_t beg = lv[L].beg, m = lv[L].end - beg;
  const int64_t chunk = (m + kLB - 1) / kLB;
  const int64_t j0 = blockIdx.x * chunk, j1 = j0 + chunk < m ? j0 + chunk : m;
  int s = 0;
  if (m <= kLB * (kT / 64) && m <= bcap) {
    // A level of few (large) cells: a wave per cell, lanes 8 d ... 8 d + 7
    // find boundary d by a 9-ary search (eight probes per step), about
    // log9 instead of log2 dependent loads.
    const int lane = threadIdx.x & 63, d = lane >> 3, r = lane & 7;
    const int sh3 = 3 * (kMaxDepth - 1 - L);
    for (int64_t base = j0; base < j1; base += kT / 64) {
      const int64_t j = base + threadIdx.x / 64;  // uniform per wave
      if (j >= j1) break;
      const int64_t c = beg + j;
      const int32_t a = C.first[c], b = a + C.n[c];
      const bool split = !(C.n[c] <= n_leaf || L == kMaxDepth);
      int32_t l = a, h = split && d > 0 ? b : a;
      // every lane of a group of eight holds the same l, h
      while (__any(l < h)) {
        const int32_t w = h - l;
        const int32_t pr = w >= 9 ? l + (int32_t)(((int64_t)w * (r + 1)) / 9) : l + r;
        const bool live = l < h && pr < h;
        const bool lt = live && (int)((key[pr] >> sh3) & 7) < d;
        const uint32_t grp = (uint32_t)(__ballot(lt) >> (lane & ~7)) & 0xffu;
        const uint32_t fal = (uint32_t)(__ballot(live && !lt) >> (lane & ~7)) & 0xffu;
        const int nt = __popc(grp);  // probes below d (a prefix of the group)
        const int32_t plast = __shfl(pr, (lane & ~7) + (nt > 0 ? nt - 1 : 0));
        const int32_t pfirst = __shfl(pr, (lane & ~7) + (nt < 8 ? nt : 7));
        if (l < h) {
          if (nt > 0) l = plast + 1;
          if (fal != 0) h = pfirst;
          else if (nt == 0) h = l;  // no live probe: nothing left
        }
      }
      const int32_t nx = __shfl_down(l, 8);
      const int32_t hi = d == 7 ? b : nx;
      const bool child = split && hi > l && r == 0;
      const int k = __popcll(__ballot(child));
      if (r == 0) bnd[8 * j + d] = l;
      s += lane == 0 ? k : 0;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) bsum[blockIdx.x] = s;
    return;
  }
  for (int64_t base = j0; base < j1; base += kT / 8) {
    const int64_t j = base + threadIdx.x / 8;
    const OctantLane o = octant_lane(C, key, beg, j, j < j1, L, n_leaf);
    int k, before;
    octant_counts(o.child, &k, &before);
    if (j < j1 && m <= bcap) bnd[8 * j + (threadIdx.x & 7)] = o.lo;
    if ((threadIdx.x & 7) == 0 && j < j1) s += k;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

// Writes level L's children in cell order; eight lanes per cell, one per
// octant, with the boundaries split_level_kernel kept (searched again for a
// level of more than bcap cells).  Every block sums the per-block children
// counts before its own (its first child's offset) and all of them (the
// level's total, for the capacity check); block 0 records the total and the
// next level's range (empty after an overflow, which it flags there).
__global__ __launch_bounds__(kT) void emit_level_kernel(Cells C, const uint64_t* __restrict__ key,
                                                        Level* __restrict__ lv, int L,
                                                        int n_leaf,
                                                        const int32_t* __restrict__ bsum,
                                                        const int32_t* __restrict__ bnd,
                                                        int64_t bcap, int64_t cap) {
  __shared__ int sh[kT / 64];
  static_assert(kLB == 2 * kT, "two block sums per thread");
  const int i0 = 2 * (int)threadIdx.x, blk = (int)blockIdx.x;
  const int s0 = bsum[i0], s1 = bsum[i0 + 1];
  const int preceding = block_sum((i0 < blk ? s0 : 0) + (i0 + 1 < blk ? s1 : 0), sh);
  const int total = block_sum(s0 + s1, sh);
  const int64_t beg = lv[L].beg, end = lv[L].end, m = end - beg;
  const bool over = lv[L].overflow || end + total > cap;
  if (blk == 0 && threadIdx.x == 0) {
    lv[L].total = over ? 0 : total;
    if (L + 1 < kMaxDepth + 2) lv[L + 1] = Level{end, over ? end : end + total, 0, over, 0};
  }
  if (over) return;
  const int64_t chunk = (m + kLB - 1) / kLB;
  const int64_t j0 = blockIdx.x * chunk, j1 = j0 + chunk < m ? j0 + chunk : m;
  int64_t carry = preceding;
  for (int64_t base = j0; base < j1; base += kT / 8) {
    const int64_t j = base + threadIdx.x / 8;
    const bool valid = j < j1;
    const OctantLane o = m <= bcap ? octant_lane_stored(C, bnd, beg, j, valid, L, n_leaf)
                                   : octant_lane(C, key, beg, j, valid, L, n_leaf);
    int k, before;
    octant_counts(o.child, &k, &before);
    const bool lead = (threadIdx.x & 7) == 0;
    int step = 0;
    const int ex = __shfl(block_exclusive(lead && valid ? k : 0, &step, sh),
                          (int)(threadIdx.x & 63) & ~7);
    const int64_t first = end + carry + ex;
    if (lead && valid && k > 0) {
      C.fc[o.c] = (int32_t)first;
      C.nc[o.c] = k;
    }
    if (o.child) {
      const int64_t ch = first + before;
      C.first[ch] = o.lo;
      C.n[ch] = o.hi - o.lo;
      C.depth[ch] = L + 1;
      C.parent[ch] = (int32_t)o.c;
      C.fc[ch] = -1;
      C.nc[ch] = 0;
    }
    carry += step;
  }
}

__global__ void gather_kernel(const float4* __restrict__ packed, const int32_t* __restrict__ perm,
                              int64_t n, float4* __restrict__ part, int32_t* __restrict__ iperm) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const int32_t p = perm[i];
  part[i] = packed[p];
  iperm[p] = (int32_t)i;
}

// The host's std::min / std::max on doubles.
__device__ __forceinline__ double hmin(double a, double b) { return b < a ? b : a; }
__device__ __forceinline__ double hmax(double a, double b) { return a < b ? b : a; }

// Box and FP64 moments of one cell, as the host computes them.  The loads of
// a leaf's particles (kMomChunk at a time) and of a cell's
// children (four at a time) are issued before their sums, so a cell costs a
// few memory round trips instead of one per particle or child.  The sums keep the
// host's order; a slot past the end repeats the last particle or child with
// weight +0, which leaves every sum and the box unchanged bit for bit (the
// sums start at +0 and the inputs are finite).
constexpr int kMomChunk = 16;
// LEAVES: cell c if it is a leaf, else nothing; otherwise cell c if it has
// children (whose moments are done), else nothing.
template <bool LEAVES>
__device__ __forceinline__ void cell_moments(const Cells& C, const float4* __restrict__ part,
                                             int64_t c, double* __restrict__ box,
                                             double* __restrict__ mp64) {
#pragma clang fp contract(off)
  double bx[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  double M = 0, sx = 0, sy = 0, sz = 0;
  double Q[6] = {0, 0, 0, 0, 0, 0};
  double com[3];
  const bool leaf = C.nc[c] == 0;
  if (leaf != LEAVES) return;
  if (LEAVES) {
    const int32_t f = C.first[c], e = f + C.n[c];
    for (int32_t i0 = f; i0 < e; i0 += kMomChunk) {
      float4 pb[kMomChunk];
#pragma unroll
      for (int k = 0; k < kMomChunk; ++k) pb[k] = part[i0 + k < e ? i0 + k : e - 1];
#pragma unroll
      for (int k = 0; k < kMomChunk; ++k) {
        const double x[3] = {pb[k].x, pb[k].y, pb[k].z};
        for (int d = 0; d < 3; ++d) {
          bx[d] = hmin(bx[d], x[d]);
          bx[3 + d] = hmax(bx[3 + d], x[d]);
        }
        const double w = i0 + k < e ? (double)pb[k].w : 0.0;
        M += w;
        sx += w * x[0];
        sy += w * x[1];
        sz += w * x[2];
      }
    }
    com[0] = sx / M;
    com[1] = sy / M;
    com[2] = sz / M;
    for (int32_t i0 = f; i0 < e; i0 += kMomChunk) {
      float4 pb[kMomChunk];
#pragma unroll
      for (int k = 0; k < kMomChunk; ++k) pb[k] = part[i0 + k < e ? i0 + k : e - 1];
#pragma unroll
      for (int k = 0; k < kMomChunk; ++k) {
        const float4 p = pb[k];
        const double d0 = p.x - com[0], d1 = p.y - com[1], d2 = p.z - com[2];
        const double w = i0 + k < e ? (double)p.w : 0.0;
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        Q[0] += w * (3 * d0 * d0 - r2);
        Q[1] += w * (3 * d1 * d1 - r2);
        Q[2] += w * (3 * d2 * d2 - r2);
        Q[3] += w * 3 * d0 * d1;
        Q[4] += w * 3 * d0 * d2;
        Q[5] += w * 3 * d1 * d2;
      }
    }
  } else {
    // Children in two batches of four (a batch's loads first, then its sums
    // in child order), which keeps the kernel at a few waves per SIMD.
    const int32_t f = C.fc[c], nk = C.nc[c];  // 1 ... 8 children
#pragma unroll 1
    for (int h = 0; h < nk; h += 4) {
      double cb[4][6], cm[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t ch = f + (h + k < nk ? h + k : nk - 1);
#pragma unroll
        for (int d = 0; d < 6; ++d) cb[k][d] = box[6 * ch + d];
#pragma unroll
        for (int d = 0; d < 4; ++d) cm[k][d] = mp64[10 * ch + d];
        if (h + k >= nk) cm[k][0] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        for (int d = 0; d < 3; ++d) {
          bx[d] = hmin(bx[d], cb[k][d]);
          bx[3 + d] = hmax(bx[3 + d], cb[k][3 + d]);
        }
        M += cm[k][0];
        sx += cm[k][0] * cm[k][1];
        sy += cm[k][0] * cm[k][2];
        sz += cm[k][0] * cm[k][3];
      }
    }
    com[0] = sx / M;
    com[1] = sy / M;
    com[2] = sz / M;
#pragma unroll 1
    for (int h = 0; h < nk; h += 4) {
      double cq[4][10];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t ch = f + (h + k < nk ? h + k : nk - 1);
#pragma unroll
        for (int d = 0; d < 10; ++d) cq[k][d] = mp64[10 * ch + d];
        if (h + k >= nk)
          for (int d = 0; d < 10; ++d) cq[k][d] = d == 0 ? 0.0 : (d < 4 ? com[d - 1] : 0.0);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double* q = cq[k];
        const double d0 = q[1] - com[0], d1 = q[2] - com[1], d2 = q[3] - com[2];
        const double w = q[0];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        Q[0] += q[4] + w * (3 * d0 * d0 - r2);
        Q[1] += q[5] + w * (3 * d1 * d1 - r2);
        Q[2] += q[6] + w * (3 * d2 * d2 - r2);
        Q[3] += q[7] + w * 3 * d0 * d1;
        Q[4] += q[8] + w * 3 * d0 * d2;
        Q[5] += q[9] + w * 3 * d1 * d2;
      }
    }
  }
  double* o = box + 6 * c;
  for (int k = 0; k < 6; ++k) o[k] = bx[k];
  double* q = mp64 + 10 * c;
  q[0] = M;
  for (int k = 0; k < 3; ++k) q[1 + k] = com[k];
  for (int k = 0; k < 6; ++k) q[4 + k] = Q[k];
}

// The leaves among cells [a, b) (all cells: leaves need only their
// particles), or the cells with children among [a, b) (one level, after the
// levels below), one thread per cell.
template <bool LEAVES>
__global__ __launch_bounds__(kT) void moments_kernel(Cells C, const float4* __restrict__ part,
                                                     int64_t a, int64_t b,
                                                     double* __restrict__ box,
                                                     double* __restrict__ mp64) {
  const int64_t c = a + (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c < b) cell_moments<LEAVES>(C, part, c, box, mp64);
}


// FP32 images of every cell: topology, boundary (centre of the tight box,
// side = largest extent; the device copy carries the leaf flag in the side's
// sign bit), walk record, moments, depth, and the learned criterion's cell features
// with the host's FP32 expressions.
__global__ void images_kernel(Cells C, int64_t nc, const double* __restrict__ box,
                              const double* __restrict__ mp64, int4* __restrict__ topo,
                              float4* __restrict__ geo_host, float4* __restrict__ geo,
                              float4* __restrict__ wrec, float4* __restrict__ mp,
                              float4* __restrict__ fcell, int32_t* __restrict__ depth,
                              int32_t* __restrict__ leaf_part) {
#pragma clang fp contract(off)
  __shared__ int sh[kT / 64];
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  // the block's leaf count (one store per block: same-address atomics
  // from every wave serialise)
  const int nl = block_sum(c < nc && C.nc[c < nc ? c : 0] == 0 ? 1 : 0, sh);
  if (threadIdx.x == 0) leaf_part[blockIdx.x] = nl;
  if (c >= nc) return;
  const int4 tp = make_int4(C.fc[c], C.nc[c], C.first[c], C.n[c]);
  topo[c] = tp;
  const int32_t dc = C.depth[c];
  depth[c] = dc;
  const double* bx = box + 6 * c;
  double l = 0;
  float g[3];
  for (int k = 0; k < 3; ++k) {
    g[k] = (float)((bx[k] + bx[3 + k]) * 0.5);
    l = hmax(l, bx[3 + k] - bx[k]);
  }
  const float lf = (float)l;
  geo_host[c] = make_float4(g[0], g[1], g[2], lf);
  const float4 gd = make_float4(g[0], g[1], g[2], tp.y == 0 ? -lf : lf);
  geo[c] = gd;
  wrec[2 * c] = gd;
  wrec[2 * c + 1] = make_float4(__int_as_float(tp.x), __int_as_float(tp.y), __int_as_float(tp.z),
                                __int_as_float(tp.w));
  const double* q = mp64 + 10 * c;
  const float m[10] = {(float)q[1], (float)q[2], (float)q[3], (float)q[0], (float)q[4],
                       (float)q[5], (float)q[6], (float)q[7], (float)q[8], (float)q[9]};
  mp[3 * c] = make_float4(m[0], m[1], m[2], m[3]);
  mp[3 * c + 1] = make_float4(m[4], m[5], m[6], m[7]);
  mp[3 * c + 2] = make_float4(m[8], m[9], 0.0f, 0.0f);
  const float mtot = (float)mp64[0];
  const float M = m[3];
  const float qn = sqrtf((m[4] * m[4] + m[5] * m[5] + m[6] * m[6]) +
                         2.0f * (m[7] * m[7] + m[8] * m[8] + m[9] * m[9]));
  float s2 = 0.0f;
  for (int k = 0; k < 3; ++k) {
    const float d = m[k] - g[k];
    s2 += d * d;
  }
  fcell[2 * c] = make_float4(log10f(M / mtot) / 3.0f, qn / (M * lf * lf),
                             (float)(bx[3] - bx[0]) / lf, (float)(bx[4] - bx[1]) / lf);
  fcell[2 * c + 1] = make_float4((float)(bx[5] - bx[2]) / lf,
                                 log2f(1.0f + (float)dc) / log2f(22.0f), sqrtf(s2) / lf,
                                 0.0f);
}

// Groups: the maximal cells with at most n_group particles, or leaves; their
// particle ranges partition the particles, so marking each group at its first
// particle and compacting orders them by first particle.
// (Also clears the nc + 1 per-group chunk counts that group_fill_kernel
// fills and the chunk scan reads.)
__global__ void group_mark_kernel(Cells C, int64_t nc, int n_group, int32_t* __restrict__ at,
                                  int32_t* __restrict__ nchunk) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c > nc) return;
  nchunk[c] = 0;
  if (c == nc) return;
  const bool cand = C.n[c] <= n_group || C.nc[c] == 0;
  const bool top = c == 0 || C.n[C.parent[c]] > n_group;
  if (cand && top) at[C.first[c]] = (int32_t)c;
}

// Group-start flags of the n particles, and a 0 at f[n] for the scan.
__global__ void flag_kernel(const int32_t* __restrict__ at, int64_t n, int32_t* __restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < n) f[i] = at[i] >= 0;
  else if (i == n) f[n] = 0;
}

__global__ void group_fill_kernel(const int32_t* __restrict__ at, const int32_t* __restrict__ f,
                                  const int32_t* __restrict__ pre, int64_t n, Cells C,
                                  const double* __restrict__ box, int32_t* __restrict__ groups,
                                  int4* __restrict__ ginfo, float4* __restrict__ gbox,
                                  int32_t* __restrict__ nchunk) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n || !f[i]) return;
  const int64_t g = pre[i];
  const int32_t c = at[i];
  groups[g] = c;
  ginfo[g] = make_int4(C.first[c], C.n[c], c, 0);
  const double* bx = box + 6 * (int64_t)c;
  gbox[2 * g] = make_float4((float)bx[0], (float)bx[1], (float)bx[2], 0.0f);
  gbox[2 * g + 1] = make_float4((float)bx[3], (float)bx[4], (float)bx[5], 0.0f);
  nchunk[g] = (C.n[c] + kChunk - 1) / kChunk;
}

__global__ void work_kernel(const int32_t* __restrict__ nchunk, const int32_t* __restrict__ pre,
                            const int32_t* __restrict__ ngp, int2* __restrict__ work) {
  const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (g >= *ngp) return;
  for (int k = 0; k < nchunk[g]; ++k) work[pre[g] + k] = make_int2((int32_t)g, k * kChunk);
}

// The build's scalars the host needs, gathered in one place on the device so
// that one copy fetches them.
struct BuildInfo {
  Level lv[kMaxDepth + 2];
  double cube[6];  // root_kernel
  int32_t bad;     // input check (bbox_kernel)
  int32_t ng, nw, leaves;
};

// The group and work-item counts and the leaf count (sum of the images
// kernel's nb per-block counts).
__global__ __launch_bounds__(kT) void counts_kernel(const int32_t* __restrict__ ngp,
                                                    const int32_t* __restrict__ nwp,
                                                    const int32_t* __restrict__ leaf_part,
                                                    int64_t nb, BuildInfo* __restrict__ info) {
  __shared__ int sh[kT / 64];
  int t = 0;
  for (int64_t i = threadIdx.x; i < nb; i += kT) t += leaf_part[i];
  t = block_sum(t, sh);
  if (threadIdx.x == 0) {
    info->ng = *ngp;
    info->nw = *nwp;
    info->leaves = t;
  }
}

// Scratch allocations of one build: fresh ones freed on every exit, or slots
// of a pool kept for the next build.
struct Scratch {
  SeqPool* pool = nullptr;
  std::vector<void*> p;
  explicit Scratch(SeqPool* sp) : pool(sp) {}
  ~Scratch() {
    for (void* q : p) hipFree(q);
  }
  template <typename T>
  T* get(int64_t count) {
    const size_t bytes = std::max<size_t>((size_t)count * sizeof(T), 256);
    if (pool) return static_cast<T*>(pool->take(bytes));
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    p.push_back(q);
    return static_cast<T*>(q);
  }
};

template <typename T>
int exclusive_sum(const T* in, T* out, int64_t n, Scratch& S, hipStream_t s) {
  size_t bytes = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)n, s) != hipSuccess) return -1;
  void* tmp = S.get<char>((int64_t)bytes);
  if (!tmp) return -2;
  return hipcub::DeviceScan::ExclusiveSum(tmp, bytes, in, out, (int)n, s) == hipSuccess ? 0 : -1;
}

}  // namespace

void* SeqPool::take(size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  if (next < ptr.size() && cap[next] >= bytes) return ptr[next++];
  // Grown slots get a quarter of headroom so that the small changes of a
  // tree from one step to the next do not reallocate them.
  const size_t want = ((bytes + bytes / 4) + 255) & ~size_t(255);
  void* q = nullptr;
  if (next < ptr.size()) {
    hipFree(ptr[next]);
    ptr[next] = nullptr;
    cap[next] = 0;
  }
  if (hipMalloc(&q, want) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (next == ptr.size()) {
    ptr.push_back(q);
    cap.push_back(want);
  } else {
    ptr[next] = q;
    cap[next] = want;
  }
  return ptr[next++];
}

SeqPool::~SeqPool() {
  for (void* q : ptr)
    if (q) hipFree(q);
}

BuildPools::~BuildPools() {
  if (pinned) hipHostFree(pinned);
}

int build_device_tree(const float* pos_in, const float* mass_in, bool inputs_on_device, int64_t n,
                      int n_leaf, int n_group, HostTree& h, DevTree& dt, DeviceArrays& out,
                      DevAlloc& alloc, void* stream, std::string& err, BuildPools* pools) {
  hipStream_t s = (hipStream_t)stream;
  if (pools) {
    pools->outer.rewind();
    pools->cells.rewind();
  }
  Scratch S(pools ? &pools->outer : nullptr);
  Scratch CS(pools ? &pools->cells : nullptr);
  auto fail = [&](const char* what) {
    err = what;
    return -1;
  };
  h = HostTree();
  h.n = n;
  h.n_leaf = n_leaf;
  h.n_group = n_group;

  // The scalars the host needs come back in two copies (after the levels,
  // after the groups), into page-locked memory kept with the pools.
  BuildInfo* info = S.get<BuildInfo>(1);
  if (!info) return fail("device allocation failed");
  BuildInfo local;
  BuildInfo* hinfo = &local;
  if (pools) {
    if (!pools->pinned && hipHostMalloc(&pools->pinned, sizeof(BuildInfo)) != hipSuccess) {
      (void)hipGetLastError();
      pools->pinned = nullptr;
    }
    if (pools->pinned) hinfo = static_cast<BuildInfo*>(pools->pinned);
  }
  auto fetch = [&](size_t off, size_t bytes) {
    return hipMemcpyAsync(reinterpret_cast<char*>(hinfo) + off, reinterpret_cast<char*>(info) + off,
                          bytes, hipMemcpyDeviceToHost, s) == hipSuccess &&
           hipStreamSynchronize(s) == hipSuccess;
  };

  // Inputs on the device (copied there, or checked there: finite positions
  // with |x| < 2^60 and finite masses > 0, as the host build requires; the
  // verdict comes back with the level counts, and every kernel before that
  // is safe on any input values).
  const float* pos = pos_in;
  const float* mass = mass_in;
  if (hipMemsetAsync(&info->bad, 0, 4, s) != hipSuccess) return fail("memset failed");
  if (!inputs_on_device) {
    float* p = S.get<float>(3 * n);
    float* q = S.get<float>(n);
    if (!p || !q) return fail("device allocation failed");
    if (hipMemcpyAsync(p, pos_in, (size_t)n * 12, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(q, mass_in, (size_t)n * 4, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail("input upload failed");
    pos = p;
    mass = q;
  }
  const bool check = inputs_on_device;  // then bbox_kernel checks them

  // Root cube (the host's rule on the device's bounding box).
  const int nbb = (int)std::min<int64_t>(1024, blocks(n));
  float* bbp = S.get<float>(6 * nbb);
  if (!bbp) return fail("device allocation failed");
  bbox_kernel<<<nbb, kT, 0, s>>>(pos, check ? mass : nullptr, n, bbp, &info->bad);
  root_kernel<<<1, kT, 0, s>>>(bbp, nbb, info->cube);

  // Keys and the stable sort (ties keep the input order).
  uint64_t* key = S.get<uint64_t>(n);
  uint64_t* key2 = S.get<uint64_t>(n);
  int32_t* idx = S.get<int32_t>(n);
  int32_t* perm = nullptr;
  if (!key || !key2 || !idx || alloc.alloc((void**)&perm, (size_t)n * 4)) return fail("device allocation failed");
  float4* packed = S.get<float4>(n);
  if (!packed) return fail("device allocation failed");
  keys_kernel<<<blocks(n), kT, 0, s>>>(pos, mass, n, info->cube, key, idx, packed);
  size_t sbytes = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, sbytes, key, key2, idx, perm, (int)n, 0, 63, s) !=
      hipSuccess)
    return fail("sort failed");
  void* stmp = S.get<char>((int64_t)sbytes);
  if (!stmp) return fail("device allocation failed");
  if (hipcub::DeviceRadixSort::SortPairs(stmp, sbytes, key, key2, idx, perm, (int)n, 0, 63, s) !=
      hipSuccess)
    return fail("sort failed");

  // Level-synchronous subdivision; cell arrays grow as needed.
  int64_t cap = 2 * n + 64;
  Cells C{};
  auto grow = [&](int64_t need) -> bool {
    if (need <= cap && C.first) return true;
    const int64_t nc2 = C.first ? std::max(need, cap + cap / 2) : need;
    Cells D{CS.get<int32_t>(nc2), CS.get<int32_t>(nc2), CS.get<int32_t>(nc2),
            CS.get<int32_t>(nc2), CS.get<int32_t>(nc2), CS.get<int32_t>(nc2)};
    if (!D.first || !D.n || !D.depth || !D.parent || !D.fc || !D.nc) return false;
    if (C.first) {
      int32_t* src[6] = {C.first, C.n, C.depth, C.parent, C.fc, C.nc};
      int32_t* dst[6] = {D.first, D.n, D.depth, D.parent, D.fc, D.nc};
      for (int k = 0; k < 6; ++k)
        if (hipMemcpyAsync(dst[k], src[k], (size_t)cap * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
          return false;
    }
    C = D;
    cap = nc2;
    return true;
  };
  if (!grow(cap)) return fail("device allocation failed");
  std::vector<int64_t> level_beg{0};
  int64_t lbeg = 0, lend = 1;
  // All levels back to back with their ranges on the device (no host round
  // trip per level); a tree that outgrows the cell arrays is redone below
  // level by level, growing them.
  {
    Level* lv = info->lv;
    int32_t* bsum = S.get<int32_t>(kLB);
    // The octant boundaries (eight per cell) go into the unsorted keys, dead
    // after the sort: levels of up to n / 4 cells keep them, larger ones
    // (only trees with very small leaves) are searched again.
    int32_t* bnd = reinterpret_cast<int32_t*>(key);
    const int64_t bcap = n / 4;
    if (!bsum) return fail("device allocation failed");
    level_init_kernel<<<1, 64, 0, s>>>(C, lv, (int32_t)n);
    // A rebuild launches the levels its previous tree had plus two, then
    // looks whether the next one is empty (an empty level still costs two
    // launches); the rest follow only if the tree turned out deeper.  The
    // copy also brings the input check and the root cube.
    int L0 = 0, L1 = kMaxDepth;
    if (pools && pools->last_levels > 0) L1 = std::min(kMaxDepth, pools->last_levels + 1);
    for (;;) {
      for (int L = L0; L <= L1; ++L) {
        split_level_kernel<<<kLB, kT, 0, s>>>(C, key2, lv, L, n_leaf, bsum, bnd, bcap);
        emit_level_kernel<<<kLB, kT, 0, s>>>(C, key2, lv, L, n_leaf, bsum, bnd, bcap, cap);
      }
      if (!fetch(0, offsetof(BuildInfo, ng))) return fail("subdivision failed");
      if (hinfo->bad & 1) return fail("positions must be finite with |x| < 2^60");
      if (hinfo->bad & 2) return fail("masses must be finite and > 0");
      if (L1 == kMaxDepth || hinfo->lv[L1 + 1].end == hinfo->lv[L1 + 1].beg) break;
      L0 = L1 + 1;
      L1 = kMaxDepth;
    }
    for (int k = 0; k < 3; ++k) h.corner[k] = hinfo->cube[k];
    h.side = hinfo->cube[3];
    bool over = false;
    for (const Level& v : hinfo->lv) over = over || v.overflow;
    if (!over) {
      int levels = 0;
      for (int L = 0; L <= kMaxDepth && hinfo->lv[L].end > hinfo->lv[L].beg; ++L) {
        h.max_level_cells = std::max(h.max_level_cells, hinfo->lv[L].end - hinfo->lv[L].beg);
        if (hinfo->lv[L].total > 0) h.max_depth = L + 1;
        level_beg.push_back(hinfo->lv[L].end);
        lbeg = lend = hinfo->lv[L].end;
        levels = L + 1;
      }
      if (pools) pools->last_levels = levels;
    }
  }
  if (lbeg < lend) {  // the arrays overflowed: level by level with growth
    const int32_t root[6] = {0, (int32_t)n, 0, -1, -1, 0};
    int32_t* rdst[6] = {C.first, C.n, C.depth, C.parent, C.fc, C.nc};
    for (int k = 0; k < 6; ++k)
      if (hipMemcpyAsync(rdst[k], &root[k], 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail("root upload failed");
  }
  for (int L = 0; lbeg < lend; ++L) {
    const int64_t m = lend - lbeg;
    if (pools) pools->level.rewind();  // the previous level's scratch is dead
    Scratch LS(pools ? &pools->level : nullptr);
    int32_t* bd = LS.get<int32_t>(9 * m);
    int32_t* nkid = LS.get<int32_t>(m + 1);
    int32_t* pre = LS.get<int32_t>(m + 1);
    if (!bd || !nkid || !pre) return fail("device allocation failed");
    split_kernel<<<blocks(m), kT, 0, s>>>(C, key2, lbeg, m, L, n_leaf, bd, nkid);
    if (hipMemsetAsync(nkid + m, 0, 4, s) != hipSuccess) return fail("memset failed");
    if (exclusive_sum(nkid, pre, m + 1, LS, s)) return fail("scan failed");
    int32_t total = 0;
    if (hipMemcpyAsync(&total, pre + m, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail("level count failed");
    if (total > 0) {
      if (!grow(lend + total)) return fail("device allocation failed");
      emit_kernel<<<blocks(m), kT, 0, s>>>(C, lbeg, lend, m, L, bd, nkid, pre);
    }
    h.max_level_cells = std::max(h.max_level_cells, m);
    if (total > 0) h.max_depth = L + 1;
    lbeg = lend;
    lend += total;
    level_beg.push_back(lbeg);  // level L spans [level_beg[L], level_beg[L + 1])
    // Fresh level scratch is freed at the end of the iteration: let the level
    // finish first (pool slots are reused in stream order instead).
    if (!pools && hipStreamSynchronize(s) != hipSuccess) return fail("subdivision failed");
  }
  const int64_t nc = lend;

  // Persistent device arrays of the tree.
  auto A = [&](void** p, size_t bytes) { return alloc.alloc(p, bytes) == 0; };
  float4* part = nullptr;
  int32_t* iperm = nullptr;
  if (!A((void**)&part, (size_t)n * 16) || !A((void**)&iperm, (size_t)n * 4))
    return fail("device allocation failed");
  gather_kernel<<<blocks(n), kT, 0, s>>>(packed, perm, n, part, iperm);

  double* box = nullptr;
  double* mp64 = nullptr;
  if (!A((void**)&box, (size_t)nc * 48) || !A((void**)&mp64, (size_t)nc * 80))
    return fail("device allocation failed");
  moments_kernel<true><<<blocks(nc), kT, 0, s>>>(C, part, 0, nc, box, mp64);
  for (int L = h.max_depth - 1; L >= 0; --L) {  // the deepest level holds only leaves
    const int64_t a = level_beg[L], b = level_beg[L + 1];
    if (b > a) moments_kernel<false><<<blocks(b - a), kT, 0, s>>>(C, part, a, b, box, mp64);
  }
  int4* topo = nullptr;
  float4 *geo_host = nullptr, *geo = nullptr, *wrec = nullptr, *mp = nullptr, *fcell = nullptr;
  int32_t* depth = nullptr;
  if (!A((void**)&topo, (size_t)nc * 16) || !A((void**)&geo_host, (size_t)nc * 16) ||
      !A((void**)&geo, (size_t)nc * 16) || !A((void**)&wrec, (size_t)nc * 32) ||
      !A((void**)&mp, (size_t)nc * 48) || !A((void**)&fcell, (size_t)nc * 32) ||
      !A((void**)&depth, (size_t)nc * 4))
    return fail("device allocation failed");
  const int64_t nbi = blocks(nc);
  int32_t* nleaf = S.get<int32_t>(nbi);
  if (!nleaf) return fail("device allocation failed");
  images_kernel<<<blocks(nc), kT, 0, s>>>(C, nc, box, mp64, topo, geo_host, geo, wrec, mp, fcell,
                                          depth, nleaf);

  // Groups and work chunks, sized by bounds known here (groups <= cells,
  // work items <= groups + n / kChunk), so that their counts come back in
  // one copy at the end.
  const int64_t ngcap = nc, nwcap = nc + n / kChunk + 1;
  int32_t* at = S.get<int32_t>(n);
  int32_t* f = S.get<int32_t>(n + 1);
  int32_t* fpre = S.get<int32_t>(n + 1);
  int32_t* nchunk = S.get<int32_t>(ngcap + 1);
  int32_t* cpre = S.get<int32_t>(ngcap + 1);
  if (!at || !f || !fpre || !nchunk || !cpre) return fail("device allocation failed");
  if (hipMemsetAsync(at, 0xff, (size_t)n * 4, s) != hipSuccess) return fail("memset failed");
  group_mark_kernel<<<blocks(nc + 1), kT, 0, s>>>(C, nc, n_group, at, nchunk);
  flag_kernel<<<blocks(n + 1), kT, 0, s>>>(at, n, f);
  if (exclusive_sum(f, fpre, n + 1, S, s)) return fail("scan failed");
  int32_t* groups = nullptr;
  int4* ginfo = nullptr;
  float4* gbox = nullptr;
  int2* work = nullptr;
  if (!A((void**)&groups, (size_t)ngcap * 4) || !A((void**)&ginfo, (size_t)ngcap * 16) ||
      !A((void**)&gbox, (size_t)ngcap * 32) || !A((void**)&work, (size_t)nwcap * 8))
    return fail("device allocation failed");
  group_fill_kernel<<<blocks(n), kT, 0, s>>>(at, f, fpre, n, C, box, groups, ginfo, gbox, nchunk);
  if (exclusive_sum(nchunk, cpre, ngcap + 1, S, s)) return fail("scan failed");
  work_kernel<<<blocks(ngcap), kT, 0, s>>>(nchunk, cpre, fpre + n, work);
  counts_kernel<<<1, kT, 0, s>>>(fpre + n, cpre + ngcap, nleaf, nbi, info);
  if (!fetch(offsetof(BuildInfo, ng), sizeof(BuildInfo) - offsetof(BuildInfo, ng)))
    return fail("group and work counts failed");
  const int64_t ng = hinfo->ng, nw = hinfo->nw;
  h.nc_dev = nc;
  h.ng_dev = ng;
  h.nw_dev = nw;
  h.n_leaves = hinfo->leaves;

  dt.part = reinterpret_cast<const float*>(part);
  dt.perm = perm;
  dt.topo = reinterpret_cast<const int32_t*>(topo);
  dt.geo = reinterpret_cast<const float*>(geo);
  dt.wrec = reinterpret_cast<const float*>(wrec);
  dt.fcell = reinterpret_cast<const float*>(fcell);
  dt.iperm = iperm;
  dt.mp = reinterpret_cast<const float*>(mp);
  dt.ginfo = reinterpret_cast<const int32_t*>(ginfo);
  dt.gbox = reinterpret_cast<const float*>(gbox);
  dt.work = reinterpret_cast<const int32_t*>(work);
  dt.n = n;
  dt.nc = nc;
  dt.ng = ng;
  dt.nw = nw;
  out.box = box;
  out.mp64 = mp64;
  out.geo_host = reinterpret_cast<const float*>(geo_host);
  out.depth = depth;
  out.groups = groups;
  return 0;
}

}  // namespace octgrav
