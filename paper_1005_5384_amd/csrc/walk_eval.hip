// Fused group walk + list evaluation (Sec. 2.2 + 2.3) for gfx950.
//
// The paper builds the lists with two walks (count, then write, with a host
// prefix sum between them) and evaluates them in separate kernels.  Here one
// 64-lane wavefront per work item (a group, or a chunk of 32 of its targets)
// walks the tree breadth-first itself, 64 candidates per step, and evaluates
// the accepted cells and opened leaves in 64-entry LDS tiles as soon as a
// tile fills.  The lists never reach HBM, the walk needs no block barrier
// (each wave owns its LDS area, wave-ordered), and with ~9 KB of LDS per
// wave 16 walks are in flight per CU, so their dependent gathers overlap
// other waves' arithmetic.  The waves are persistent: work items (whose
// costs differ by orders of magnitude) are handed out through per-XCD
// counters, which removed the tail of the one-block-per-item launch (11 %).
//
// The walk is the same as the two-pass walk (same test, same breadth-first
// order, ballot compaction in lane order), so the cell and leaf lists are
// identical; an export mode writes them at offsets from the count walk for
// the parity tests.  Each candidate costs one 32-byte gather (boundary +
// topology).  The frontier FIFO holds one entry per opened cell (its
// children are consecutive cells): a step takes the next 64 children of the
// queued entries, finding each lane's entry with one mark per entry in LDS
// and a ballot, so an opened cell costs one store instead of one per child,
// and a queue entry stands for up to eight candidates.  Evaluation: the wave splits into S = floor(64 / n) slices of n
// lanes; every slice holds all n targets and takes every S-th source of a
// tile; plain FP32 per tile is folded into Neumaier pairs; slices are
// combined in slice order.
//
// A work item whose frontier outgrows its LDS queue aborts before writing any
// result and is redone by the next tier: 512-entry LDS queues, then
// 2048-entry LDS queues, then queues in global memory sized so that they
// cannot overflow.
//
// Learned acceptance criterion (LEARNED): candidates the test at theta_lo
// accepts are accepted, those the test at theta_hi opens are opened, and for
// the band in between the wave computes the 12 features of its band lanes,
// stages them as consecutive rows in LDS and runs the network on the matrix
// cores over ceil(rows / 16) tiles; a candidate is accepted iff the predicted
// log10 error is at most log10 tau_pair.  The accepted band candidates' predicted errors add up
// (FP64, sqrt of the sum of squares) into the group's budget; a work item
// whose group exceeds it drops its accumulators and walks again with the
// call's theta.  Every work item of a group makes the same decisions (same
// candidates, same network arithmetic, same reduction order).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "mlp_device.h"
#include "octgrav_internal.h"

namespace octgrav {
namespace {

using namespace dev;

constexpr int kLanes = 64;
constexpr int kTileW = 64;   // sources per tile
constexpr int kRingW = 128;  // pending cells / leaves (two tiles)

// Frontier entry: x = first child << 3 | (children - 1) (cell ids < 2^29),
// y = position of the first child in the item's candidate sequence.
template <int QCAP>
struct WShared {
  int2 q[QCAP];
  int cring[kRingW];
  int2 lring[kRingW];  // (first particle, n particles) of opened leaves
  float4 tile[3 * kTileW];
  int pre[kTileW + 1];
  int lfirst[kTileW];
};

// Orders this wave's LDS accesses: lanes read what other lanes of the same
// wave wrote before (LDS executes a wave's instructions in order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS frontier queue of one wave.
struct LQueue {
  int2* p;
  __device__ int2 get(uint32_t i) const { return p[i]; }
  __device__ void put(uint32_t i, int x, int y) const { p[i] = make_int2(x, y); }
};

template <bool PLAIN, typename SH>
struct WItem {
  const DevTree& T;
  SH& sh;
  float eps2;
  int lane, nt, S, slice;
  bool active, do_eval;
  float4 xi;
  Sum4 acc4;
  int64_t nsrc = 0;

  __device__ void flush_cells(uint32_t start, int cnt) {
    if (!do_eval) return;
    const float4* mp = reinterpret_cast<const float4*>(T.mp);
    if (lane < cnt) {
      const int64_t id = sh.cring[(start + lane) & (kRingW - 1)];
      const float4 a = mp[3 * id], b = mp[3 * id + 1], c = mp[3 * id + 2];
      sh.tile[lane] = a;
      sh.tile[kTileW + lane] = b;
      sh.tile[2 * kTileW + lane] = c;
    }
    wave_lds_sync();
    if (active) {
      float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
      const float4* t0 = sh.tile;
      const float4* t1 = sh.tile + kTileW;
      const float4* t2 = sh.tile + 2 * kTileW;
      strided2(slice, cnt, S, [&](int j) { pc_term(xi, t0[j], t1[j], t2[j], eps2, ax, ay, az, ph); });
      acc4.template fold<PLAIN>(ax, ay, az, ph);
    }
    wave_lds_sync();
  }

  __device__ void flush_leaves(uint32_t start, int lc) {
    int ln = 0;
    if (lane < lc) {
      const int2 fl = sh.lring[(start + lane) & (kRingW - 1)];
      sh.lfirst[lane] = fl.x;
      ln = fl.y;
    }
    int incl = ln;
#pragma unroll
    for (int o = 1; o < kLanes; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    const int total = __shfl(incl, kLanes - 1);
    nsrc += total;
    if (!do_eval) return;
    if (lane < lc) sh.pre[lane] = incl - ln;
    if (lane == 0) sh.pre[lc] = total;
    wave_lds_sync();
    const float4* part = reinterpret_cast<const float4*>(T.part);
    for (int u0 = 0; u0 < total; u0 += kTileW) {
      const int cnt = min(kTileW, total - u0);
      if (lane < cnt) {
        const int u = u0 + lane;
        int lo = 0, hi = lc;  // pre[lo] <= u < pre[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (sh.pre[mid] <= u) lo = mid;
          else hi = mid;
        }
        sh.tile[lane] = part[sh.lfirst[lo] + (u - sh.pre[lo])];
      }
      wave_lds_sync();
      if (active) {
        float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
        const float4* t0 = sh.tile;
        strided2(slice, cnt, S, [&](int j) { pp_term(xi, t0[j], eps2, ax, ay, az, ph); });
        acc4.template fold<PLAIN>(ax, ay, az, ph);
      }
      wave_lds_sync();
    }
  }
};

enum : int { kOverflow = 0, kDone = 1, kFallBack = 2 };

// Walks and evaluates work item w with one wave.  Returns kOverflow
// (uniformly, before writing any result) if the frontier outgrows the queue;
// with LEARNED, kFallBack (nothing written but the trace) if the group's
// budget is exceeded, *nband = band candidates visited.  cw is the value of
// cnt[g].w written by a walk with the theta test.
template <bool PLAIN, bool LEARNED, typename SH, typename Q>
__device__ int walk_eval_item(const DevTree& T, const WalkBufs& B, SH& sh, int64_t w,
                              float th2, float eps2, float* __restrict__ acc,
                              float* __restrict__ pot, Q q, uint32_t qmask, bool gmem_q,
                              bool do_eval, int cw, int* nband_out, const MlpView* mv) {
  const int lane = threadIdx.x & (kLanes - 1);
  // Per-item constants; with the learned criterion they are held in scalar
  // registers (its network needs the vector registers).
  auto U = [](auto v) {
    if constexpr (LEARNED) return uni(v);
    else return v;
  };
  const int2 wk0 = reinterpret_cast<const int2*>(T.work)[w];
  const int2 wk = make_int2(U(wk0.x), U(wk0.y));
  const int64_t g = wk.x;
  const int4 gi = U(reinterpret_cast<const int4*>(T.ginfo)[g]);
  const float4* gbox = reinterpret_cast<const float4*>(T.gbox);
  const float4 gmin = U(gbox[2 * g]), gmax = U(gbox[2 * g + 1]);
  const float4* rec = reinterpret_cast<const float4*>(T.wrec);

  WItem<PLAIN, SH> it{T, sh, eps2};
  it.lane = lane;
  it.nt = min(kChunk, gi.y - wk.y);
  it.S = kLanes / it.nt;
  it.slice = lane / it.nt;
  it.active = it.slice < it.S;
  it.do_eval = do_eval;
  const int first = gi.x + wk.y;
  it.xi = reinterpret_cast<const float4*>(T.part)[first + lane % it.nt];
  it.acc4.zero();

  const bool exp = B.export_lists && wk.y == 0;
  // learned criterion state
  const bool trace = LEARNED && B.tr_s != nullptr && wk.y == 0;
  const int64_t trb = trace ? U(B.tr_off[g]) : 0, tre = trace ? U(B.tr_off[g + 1]) : 0;
  const MacGroup mg = mac_group(gmin, gmax);
  double sum2 = 0.0;
  int nband = 0;
  const int64_t xcb = exp ? U(B.c_off[g]) : 0, xce = exp ? U(B.c_off[g + 1]) : 0;
  const int64_t xlb = exp ? U(B.l_off[g]) : 0, xle = exp ? U(B.l_off[g + 1]) : 0;

  // Frontier: entries [rhead, rtail) of q; candidates [vhead, vtail) of the
  // item's breadth-first sequence (the entry at rhead may be partly taken).
  uint32_t rhead = 0, rtail = 0, vhead = 0, vtail = 0;
  uint32_t chead = 0, ctail = 0, lhead = 0, ltail = 0;
  const int4 root = reinterpret_cast<const int4*>(rec)[1];
  if (root.y == 0) {  // the root is a leaf: its particles are the whole list
    if (lane == 0) {
      sh.lring[0] = make_int2(root.z, root.w);
      if (exp && xlb < xle) B.l_ids[xlb] = 0;
    }
    ltail = 1;
  } else {
    if (lane == 0) q.put(0, (root.x << 3) | (root.y - 1), 0);
    rtail = 1;
    vtail = (uint32_t)root.y;
  }
  // Each step marks, in sh.lfirst, the lane at which each taken entry's
  // children begin, with a value no earlier step of this item used
  // (-1 - vhead) and that no particle index equals.
  sh.lfirst[lane] = 0;
  if (gmem_q) __threadfence_block();  // queue stores complete before other lanes read
  wave_lds_sync();

  // Candidate of each lane for the next min(64, vtail - vh) candidates from
  // position vh, whose entry is rh; *used = entries that window uses up.
  auto take = [&](uint32_t rh, uint32_t vh, uint32_t* used) {
    const uint32_t nent = min((uint32_t)kLanes, rtail - rh);
    const uint32_t navail = min((uint32_t)kLanes, vtail - vh);
    const bool inq = (uint32_t)lane < nent;
    int2 e = make_int2(0, 0);
    if (inq) e = q.get((rh + lane) & qmask);
    // First lane of this entry's children in the window (<= 0 for a partly
    // taken head entry) and one past its last.
    const int s0 = (int)((uint32_t)e.y - vh);
    const int s1 = s0 + (int)((uint32_t)e.x & 7u) + 1;
    const bool inwin = inq && s0 < kLanes;
    const int stamp = -1 - (int)vh;
    if (inwin) sh.lfirst[max(s0, 0)] = stamp;
    wave_lds_sync();
    const bool mark = sh.lfirst[lane] == stamp;
    const uint64_t mM = __ballot(mark);
    const int own = rank_below(mM) + (mark ? 0 : -1);  // entry of this lane's candidate
    const int cfirst = __shfl((int)((uint32_t)e.x >> 3) - s0, own);
    *used = (uint32_t)__popcll(__ballot(inwin && s1 <= (int)navail));
    // lanes past the candidates read the root's record
    return (uint32_t)lane < navail ? cfirst + lane : 0;
  };
  // Learned criterion: a step that runs the network also scores the next
  // step's band candidates when all of them are queued already (they come
  // before anything this step queues), so one network call serves two steps
  // with fuller tiles; the next step then reuses the candidates, tests and
  // scores kept here.
  bool have_next = false;
  int c_next = 0;
  float y_next = 0.0f;
  uint32_t used_next = 0;
  uint64_t mO_next = 0, mB_next = 0;

  while (vhead < vtail) {
    const uint32_t navail = min((uint32_t)kLanes, vtail - vhead);
    const bool valid = (uint32_t)lane < navail;
    int c;
    uint32_t used;
    if (LEARNED && have_next) {
      c = c_next;
      used = used_next;
    } else {
      c = take(rhead, vhead, &used);
    }
    rhead += used;
    vhead += navail;

    const int4 tp = reinterpret_cast<const int4*>(rec)[2 * (int64_t)c + 1];
    bool op;
    if (LEARNED) {
      bool olo, band, accb = false;
      uint64_t mB;
      float yh = 0.0f;
      uint16_t* xs = reinterpret_cast<uint16_t*>(sh.tile);
      if (have_next) {
        have_next = false;
        olo = (mO_next >> lane) & 1;
        band = (mB_next >> lane) & 1;
        mB = mB_next;
        yh = y_next;
      } else {
        const float4* fc = reinterpret_cast<const float4*>(T.fcell);
        {
          const float4 ge = rec[2 * (int64_t)c];
          const float4 fc0 = fc[2 * (int64_t)c], fc1 = fc[2 * (int64_t)c + 1];
          olo = valid && open_cell(gmin, gmax, ge, B.mac_lo2);
          band = olo && !open_cell(gmin, gmax, ge, B.mac_hi2);
          mB = __ballot(band);
          // Band lanes stage their features as consecutive rows.
          if (band) {
            float f[kMlpIn];
            mac_features(mg, ge, fc0, fc1, f);
            mlp_stage(xs, kXsLd, rank_below(mB), f);
          }
        }
        if (mB) {
          const int ra = __popcll(mB);
          int rows = ra;
          if (vtail - vhead >= (uint32_t)kLanes) {  // the next step's 64 candidates are queued
            uint32_t u2;
            const int c2 = take(rhead, vhead, &u2);
            const float4 ge = rec[2 * (int64_t)c2];
            const float4 fc0 = fc[2 * (int64_t)c2], fc1 = fc[2 * (int64_t)c2 + 1];
            const bool olo2 = open_cell(gmin, gmax, ge, B.mac_lo2);
            const bool band2 = olo2 && !open_cell(gmin, gmax, ge, B.mac_hi2);
            const uint64_t mB2 = __ballot(band2);
            if (ra + __popcll(mB2) <= kLanes) {  // every row's score lands in its own lane
              if (band2) {
                float f[kMlpIn];
                mac_features(mg, ge, fc0, fc1, f);
                mlp_stage(xs, kXsLd, ra + rank_below(mB2), f);
              }
              rows += __popcll(mB2);
              have_next = true;
              c_next = c2;
              used_next = u2;
              mO_next = __ballot(olo2);
              mB_next = mB2;
            }
          }
          // The network runs on ceil(rows / 16) tiles; lane l receives row l's output.
          wave_lds_sync();
          const float yrow = mlp_scores(*mv, xs, kXsLd, lane, (rows + 15) >> 4);
          wave_lds_sync();
          yh = __shfl(yrow, rank_below(mB));
          if (have_next) y_next = __shfl(yrow, ra + rank_below(mB_next));
        }
      }
      if (mB) {
        accb = band && yh <= B.mac_ltau;
        // 10^(2 y) = 2^(2 log2(10) y) on the FP32 exp unit; summed in FP64
        if (accb) sum2 += (double)__builtin_amdgcn_exp2f(yh * 6.64385618977472f);
        if (band && trace) {
          const int64_t k = trb + nband + rank_below(mB);
          if (k < tre) {
            B.tr_c[k] = c;
            B.tr_s[k] = yh;
          }
        }
        nband += __popcll(mB);
      }
      op = olo && !accb;
    } else {
      const float4 ge = rec[2 * (int64_t)c];
      op = valid && open_cell(gmin, gmax, ge, th2);
    }
    const bool toC = valid && !op, toL = op && tp.y == 0, toQ = op && tp.y != 0;
    const uint64_t mC = __ballot(toC), mL = __ballot(toL), mQ = __ballot(toQ);
    // Queue position of each opened cell's first child: prefix of the
    // children counts (1..8) over the opened lanes, one ballot per bit.
    const int nch = toQ ? tp.y : 0;
    int preN = 0, totN = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint64_t m = __ballot((nch >> b) & 1);
      preN += rank_below(m) << b;
      totN += __popcll(m) << b;
    }
    const uint32_t nq = (uint32_t)__popcll(mQ);
    if ((rtail + nq) - rhead > qmask + 1) return kOverflow;
    if (toC) {
      const uint32_t k = ctail + rank_below(mC);
      sh.cring[k & (kRingW - 1)] = c;
      if (exp && xcb + k < xce) B.c_ids[xcb + k] = c;
    }
    if (toL) {
      const uint32_t k = ltail + rank_below(mL);
      sh.lring[k & (kRingW - 1)] = make_int2(tp.z, tp.w);
      if (exp && xlb + k < xle) B.l_ids[xlb + k] = c;
    }
    if (toQ) q.put((rtail + rank_below(mQ)) & qmask, (tp.x << 3) | (tp.y - 1), (int)(vtail + preN));
    ctail += __popcll(mC);
    ltail += __popcll(mL);
    rtail += nq;
    vtail += (uint32_t)totN;
    if (gmem_q) __threadfence_block();
    wave_lds_sync();
    if (ctail - chead >= (uint32_t)kTileW) {
      it.flush_cells(chead, kTileW);
      chead += kTileW;
    }
    if (ltail - lhead >= (uint32_t)kTileW) {
      it.flush_leaves(lhead, kTileW);
      lhead += kTileW;
    }
  }
  while (ctail != chead) {
    const int n = (int)min((uint32_t)kTileW, ctail - chead);
    it.flush_cells(chead, n);
    chead += n;
  }
  while (ltail != lhead) {
    const int n = (int)min((uint32_t)kTileW, ltail - lhead);
    it.flush_leaves(lhead, n);
    lhead += n;
  }

  if (LEARNED) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum2 += __shfl_xor(sum2, o);
    if (sqrt(sum2) > B.mac_budget) {
      *nband_out = nband;
      return kFallBack;
    }
    cw = 2 * nband;
  }
  if (lane == 0 && wk.y == 0)  // per-group counts; the totals are reduced afterwards
    reinterpret_cast<int4*>(B.cnt)[g] = make_int4((int)ctail, (int)ltail, (int)it.nsrc, cw);
  if (!do_eval) return kDone;

  // Combine the slices of each target in slice order.
  float* red = reinterpret_cast<float*>(sh.tile);  // [64][8] floats
  if (it.active) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      red[lane * 8 + k] = it.acc4.s[k];
      red[lane * 8 + 4 + k] = it.acc4.c[k];
    }
  }
  wave_lds_sync();
  if (lane < it.nt) {
    float s[4] = {0.f, 0.f, 0.f, 0.f}, cc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int sl = 0; sl < it.S; ++sl) {
      const float* r = red + (sl * it.nt + lane) * 8;
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
    const int64_t o = T.perm[first + lane];
    acc[3 * o + 0] = s[0] + cc[0];
    acc[3 * o + 1] = s[1] + cc[1];
    acc[3 * o + 2] = s[2] + cc[2];
    if (pot) pot[o] = s[3] + cc[3];
  }
  wave_lds_sync();
  return kDone;
}

// One work item, with the theta re-walk of a group over its budget.
template <bool PLAIN, bool LEARNED, typename SH, typename Q>
__device__ int walk_eval_one(const DevTree& T, const WalkBufs& B, SH& sh, int64_t w, float th2,
                             float eps2, float* acc, float* pot, Q q, uint32_t qmask, bool gmem_q,
                             bool do_eval, const MlpView* mv) {
  int nb = 0;
  const int st = walk_eval_item<PLAIN, LEARNED>(T, B, sh, w, th2, eps2, acc, pot, q, qmask, gmem_q,
                                                do_eval, 0, &nb, mv);
  if (!LEARNED || st != kFallBack) return st;
  return walk_eval_item<PLAIN, false>(T, B, sh, w, th2, eps2, acc, pot, q, qmask, gmem_q, do_eval,
                                      2 * nb + 1, &nb, mv);
}

// Next work index from a shared counter, one atomic per wave.
__device__ __forceinline__ int take_work(int32_t* ctr, int lane) {
  int k = 0;
  if (lane == 0) k = atomicAdd(ctr, 1);
  return uni(__shfl(k, 0));
}

// Persistent blocks of NW independent waves (with the learned criterion
// they share one LDS copy of the network, loaded once per block).  Without
// FROM_LIST each XCD owns a contiguous (Morton) range of work items, handed
// out one at a time through a per-XCD counter (work items differ a lot in
// cost), and a wave whose XCD's range is exhausted helps the other XCDs;
// with FROM_LIST the items are the *src_n entries of src (the overflows of
// an earlier tier), handed out through one counter.  Items whose frontier
// outgrows this kernel's LDS queue are appended to (ovl, ovn).  Blocks of 16
// waves (the learned criterion: one network copy per CU) are held to 128
// VGPRs so that four waves per SIMD fit; the few registers this spills are
// outside the loops (the same lists took 13 % longer than in the opening-
// angle kernel at three waves per SIMD, 6 % at four).
template <bool PLAIN, int QCAP, bool LEARNED, int NW, bool FROM_LIST>
__global__ __launch_bounds__(NW * kLanes) __attribute__((amdgpu_waves_per_eu(NW == 16 ? 4 : 1)))
void walk_eval_persistent_kernel(
    DevTree T, WalkBufs B, float th2, float eps2, float* acc, float* pot, int do_eval,
    const int32_t* src, const int32_t* src_n, int32_t* ovl, int32_t* ovn) {
  __shared__ WShared<QCAP> shw[NW];
  __shared__ std::conditional_t<LEARNED, MlpLds, char> ml;
  if (FROM_LIST && *src_n == 0) return;
  MlpView V{};
  if constexpr (LEARNED) {
    mlp_load_lds(ml, B.mlp, threadIdx.x, blockDim.x);
    __syncthreads();
    V = mlp_lds(ml);
  }
  const int wv = threadIdx.x / kLanes, lane = threadIdx.x & (kLanes - 1);
  // lds_qcap counts candidates; an entry holds up to eight
  const uint32_t qmask = (uint32_t)min(B.lds_qcap / 8, QCAP) - 1;
  const LQueue q{shw[wv].q};
  if constexpr (FROM_LIST) {
    for (;;) {
      const int k = take_work(B.wctr + 64 * 8, lane);
      if (k >= *src_n) break;
      const int32_t w = src[k];
      if (walk_eval_one<PLAIN, LEARNED>(T, B, shw[wv], w, th2, eps2, acc, pot, q, qmask, false,
                                        do_eval != 0, &V) == kOverflow &&
          lane == 0)
        ovl[atomicAdd(ovn, 1)] = w;
    }
  } else {
    const int64_t per = (T.nw + 7) / 8;
    for (int s = 0; s < 8; ++s) {
      const int x = (blockIdx.x + s) & 7;
      const int64_t lo = x * per, n = max((int64_t)0, min(per, T.nw - lo));
      for (;;) {
        const int k = take_work(B.wctr + 64 * x, lane);
        if (k >= n) break;
        const int64_t w = lo + k;
        if (walk_eval_one<PLAIN, LEARNED>(T, B, shw[wv], w, th2, eps2, acc, pot, q, qmask, false,
                                          do_eval != 0, &V) == kOverflow &&
            lane == 0)
          ovl[atomicAdd(ovn, 1)] = (int32_t)w;
      }
    }
  }
}

// Global-memory queues: written and read by different lanes of one wave, so
// they are accessed as volatile (no stale L1 copies) and fenced.  The two
// words of entry i sit at p[i] and p[cap + i].
struct GQueue {
  volatile int32_t* p;
  int64_t cap;
  __device__ int2 get(uint32_t i) const { return make_int2(p[i], p[cap + i]); }
  __device__ void put(uint32_t i, int x, int y) const {
    p[i] = x;
    p[cap + i] = y;
  }
};

// Last tier: the *src_n items of src with global-memory frontier queues of
// 2 x (widest tree level) entries, which a breadth-first FIFO cannot exceed
// (its candidates span at most two consecutive levels, and every queued
// entry holds at least one of them).
template <bool PLAIN, bool LEARNED>
__global__ __launch_bounds__(kLanes) void walk_eval_fallback_kernel(DevTree T, WalkBufs B,
                                                                    float th2, float eps2,
                                                                    float* acc, float* pot,
                                                                    int do_eval,
                                                                    const int32_t* src,
                                                                    const int32_t* src_n) {
  __shared__ WShared<64> sh;
  __shared__ std::conditional_t<LEARNED, MlpLds, char> ml;
  const int n = *src_n;
  if (n == 0) return;
  MlpView V{};
  if constexpr (LEARNED) {
    mlp_load_lds(ml, B.mlp, threadIdx.x, blockDim.x);
    __syncthreads();
    V = mlp_lds(ml);
  }
  GQueue q{B.gq + (int64_t)blockIdx.x * 2 * B.gq_cap, B.gq_cap};
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int st = walk_eval_one<PLAIN, LEARNED>(T, B, sh, src[i], th2, eps2, acc, pot, q,
                                                 (uint32_t)(B.gq_cap - 1), true, do_eval != 0, &V);
    if (st == kOverflow && threadIdx.x == 0)
      atomicOr(reinterpret_cast<unsigned long long*>(&B.tot[5]), 1ull);
  }
}

__global__ void fused_init_kernel(WalkBufs B) {
  if (threadIdx.x < 8) B.tot[threadIdx.x] = 0;
  if (threadIdx.x < 9) B.wctr[64 * threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    *B.ovf_count = 0;
    *B.ovf_count2 = 0;
    B.c_off[0] = 0;  // base of an offsets scan of the counts this walk writes
    B.l_off[0] = 0;
  }
}

}  // namespace

int launch_walk_eval(const DevTree& T, const WalkBufs& B, float theta, float eps, bool plain,
                     bool do_eval, float* acc, float* pot, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const float th2 = theta * theta, eps2 = eps * eps;
  fused_init_kernel<<<1, 64, 0, s>>>(B);
  // The breadth-first FIFO holds about two tree levels of the group's walk,
  // which grow like theta^-3, as entries of up to eight children: 512 entries
  // (4 KB) held every walk of the 2^20 Plummer sphere and the 4M clumps at
  // theta 0.3 ... 0.5.  Tiers: 512-entry LDS queues (16 waves per CU), then
  // the overflows with 2048-entry LDS queues (one wave per block, 7 per CU),
  // then global-memory queues.
  const bool learned = B.mlp != nullptr;
  auto go = [&](auto plain_tag, auto learned_tag) {
    constexpr bool P = decltype(plain_tag)::value, L = decltype(learned_tag)::value;
    if constexpr (L)  // one block of 16 waves per CU (16 x 9 KB frontiers + 12 KB network,
                      // 159.6 KB of LDS), four per SIMD at <= 128 VGPRs
      walk_eval_persistent_kernel<P, 512, L, 16, false><<<8 * 32, 16 * kLanes, 0, s>>>(
          T, B, th2, eps2, acc, pot, do_eval, nullptr, nullptr, B.ovf_list, B.ovf_count);
    else  // 4 blocks of 4 waves per CU
      walk_eval_persistent_kernel<P, 512, L, 4, false><<<8 * 128, 4 * kLanes, 0, s>>>(
          T, B, th2, eps2, acc, pot, do_eval, nullptr, nullptr, B.ovf_list, B.ovf_count);
    walk_eval_persistent_kernel<P, 2048, L, 1, true><<<8 * 224, kLanes, 0, s>>>(
        T, B, th2, eps2, acc, pot, do_eval, B.ovf_list, B.ovf_count, B.ovf_list2, B.ovf_count2);
    walk_eval_fallback_kernel<P, L><<<B.gq_waves, kLanes, 0, s>>>(T, B, th2, eps2, acc, pot, do_eval,
                                                                 B.ovf_list2, B.ovf_count2);
  };
  if (learned) {
    if (plain) go(std::true_type{}, std::true_type{});
    else go(std::false_type{}, std::true_type{});
  } else {
    if (plain) go(std::true_type{}, std::false_type{});
    else go(std::false_type{}, std::false_type{});
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace octgrav
