// C ABI of the library (declared in include/octgrav.h): argument checks,
// ownership of host and device memory, and the order of the device phases
// of one force call (Sec. 2: count walk, offsets, write walk, evaluation),
// followed by the FP64 diagnostics.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <new>
#include <memory>
#include <string>
#include <vector>

#include "octgrav.h"
#include "octgrav_internal.h"

using namespace octgrav;

namespace octgrav {
int fallback_waves();
}

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Set by the environment variable OCTGRAV_FAIL_ALLOC=1 (test-only fault
// injection): every device allocation of the library fails.
bool alloc_fault() {
  const char* v = std::getenv("OCTGRAV_FAIL_ALLOC");
  return v && v[0] == '1';
}

// OCTGRAV_DEBUG=1 traces each force call's path decisions on stderr.
bool debug_trace() {
  static const bool on = [] {
    const char* v = std::getenv("OCTGRAV_DEBUG");
    return v && v[0] == '1';
  }();
  return on;
}

// Set by OCTGRAV_LDS_QUEUE=<power of two> (test-only): caps the walks' LDS
// frontier queues so that groups overflow into the global-memory fallback
// walks.  Unset, the kernels use their full queues.
int lds_queue_entries() {
  const char* v = std::getenv("OCTGRAV_LDS_QUEUE");
  int q = v ? std::atoi(v) : (1 << 20);
  if (q < 64 || (q & (q - 1))) q = 1 << 20;
  return q;
}

}  // namespace

// Network of the learned criterion: FP32 master parameters, Adam moments,
// the last gradient, the packed BF16 inference image and training scratch.
struct octgrav_mlp {
  hipStream_t stream = nullptr;
  void *P = nullptr, *mom1 = nullptr, *mom2 = nullptr, *grad = nullptr, *pk = nullptr,
       *d_loss = nullptr, *scratch = nullptr;
  int64_t scratch_b = 0;
  std::vector<void*> allocs;

  ~octgrav_mlp() {
    for (void* p : allocs) hipFree(p);
  }
  int alloc(void** p, size_t bytes) {
    if (alloc_fault() || hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return fail(OCTGRAV_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    allocs.push_back(*p);
    return OCTGRAV_OK;
  }
  // Training scratch for batches of up to b samples (activations, gradients
  // and the partial gradient sums of launch_mlp_loss_grad).
  int reserve(int64_t b) {
    if (b <= scratch_b) return OCTGRAV_OK;
    if (scratch) {
      hipFree(scratch);
      allocs.erase(std::find(allocs.begin(), allocs.end(), scratch));
      scratch = nullptr;
      scratch_b = 0;
    }
    if (int rc = alloc(&scratch, (size_t)mlp_train_scratch_floats(b) * 4))
      return rc;
    scratch_b = b;
    return OCTGRAV_OK;
  }
};

struct octgrav_tree : DevAlloc {
  HostTree h;
  bool dev = false;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  DevTree dt{};
  WalkBufs wb{};
  double* d_diag_part = nullptr;
  double* d_diag = nullptr;
  bool have_diag = false;
  bool counts_valid = false;
  hipEvent_t ev[6] = {};
  double timings[6] = {0, 0, 0, 0, 0, 0};
  // Pipelined two-pass path: a second stream for the evaluation of batch b
  // while the walks of batch b+1 run on the handle's stream.
  static constexpr int kBatches = 8;
  hipStream_t eval_stream = nullptr;
  hipEvent_t bev[kBatches + 2] = {};
  std::vector<int64_t> gwork;  // [ng+1] first work item of each group
  int64_t slot_c = 0, slot_l = 0;  // per-group list slots of the pipelined path (0 = unsized)
  // Learned acceptance criterion: a private copy of the network's packed image.
  void* d_mlp = nullptr;
  bool learned = false;
  // Walk records of the centre-of-mass offset test, for the theta they were
  // made for (made on first use, remade when theta changes).
  float* d_wrec_com = nullptr;
  float com_theta = -1.0f;
  // Handles rebuilt in place (time integration) take their device buffers
  // from pools that the next rebuild reuses.
  std::unique_ptr<SeqPool> pool;
  std::unique_ptr<BuildPools> build_pools;

  int64_t* tot_host = nullptr;  // page-locked copy of the totals (read after every call)

  ~octgrav_tree() {
    if (tot_host) hipHostFree(tot_host);
    for (void* p : allocs) hipFree(p);
    for (hipEvent_t e : ev)
      if (e) hipEventDestroy(e);
    for (hipEvent_t e : bev)
      if (e) hipEventDestroy(e);
    if (eval_stream) hipStreamDestroy(eval_stream);
  }

  int alloc(void** p, size_t bytes) override { return dalloc(p, bytes); }

  // Device-built trees keep the FP64 boxes and moments, the boundary image,
  // the particle order and the FP32 moments on the device until an export
  // asks for them.
  DeviceArrays darr;
  bool host_partial = false;

  int fetch_host_arrays() {
    if (!host_partial) return OCTGRAV_OK;
    const int64_t n = h.n, nc = h.n_cells();
    const int64_t ng = h.n_groups(), nw = h.n_work();
    h.perm.resize(n);
    h.depth.resize(nc);
    h.groups.resize(ng);
    h.work.resize((size_t)nw * 2);
    h.topo.resize((size_t)nc * 4);
    h.geo.resize((size_t)nc * 4);
    h.mp.resize((size_t)nc * 12);
    h.mp64.resize((size_t)nc * 10);
    h.box.resize((size_t)nc * 6);
    if (hipMemcpy(h.perm.data(), dt.perm, (size_t)n * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(h.topo.data(), dt.topo, (size_t)nc * 16, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(h.geo.data(), darr.geo_host, (size_t)nc * 16, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(h.mp.data(), dt.mp, (size_t)nc * 48, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(h.mp64.data(), darr.mp64, (size_t)nc * 80, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(h.box.data(), darr.box, (size_t)nc * 48, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(h.depth.data(), darr.depth, (size_t)nc * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        (ng > 0 && hipMemcpy(h.groups.data(), darr.groups, (size_t)ng * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
        (nw > 0 && hipMemcpy(h.work.data(), dt.work, (size_t)nw * 8, hipMemcpyDeviceToHost) != hipSuccess))
      return fail(OCTGRAV_EHIP, "tree copy-back failed");
    host_partial = false;
    return OCTGRAV_OK;
  }

  int dalloc(void** p, size_t bytes) {
    if (alloc_fault()) return fail(OCTGRAV_ENOMEM, "device allocation failed (injected)");
    if (pool) {
      *p = pool->take(bytes);
      if (!*p) return fail(OCTGRAV_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
      return OCTGRAV_OK;
    }
    if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(OCTGRAV_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    allocs.push_back(*p);
    return OCTGRAV_OK;
  }

  void dfree(void* p) {
    if (pool) return;  // pool slots live until the handle is freed
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) {
      hipFree(p);
      allocs.erase(it);
    }
  }

  template <typename T>
  int upload(const std::vector<T>& v, const T** out) {
    void* p = nullptr;
    if (int rc = dalloc(&p, v.size() * sizeof(T))) return rc;
    if (!v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
      return fail(OCTGRAV_EHIP, "hipMemcpy (tree upload) failed");
    *out = (const T*)p;
    return OCTGRAV_OK;
  }

  int to_device() {
    const int64_t n = h.n, nc = h.n_cells(), ng = h.n_groups(), nw = h.n_work();
    dt.n = n;
    dt.nc = nc;
    dt.ng = ng;
    dt.nw = nw;
    int rc;
    // Device boundary sides carry the leaf flag in their sign bit (the
    // opening test squares the side, so its decisions are unchanged).
    std::vector<float> geo_dev(h.geo);
    for (int64_t c = 0; c < nc; ++c)
      if (h.topo[4 * c + 1] == 0) geo_dev[4 * c + 3] = -geo_dev[4 * c + 3];
    // Walk record: the boundary and the topology of a cell in one 32-byte
    // line, so one gather serves a candidate's test and its expansion.
    std::vector<float> wrec((size_t)nc * 8);
    for (int64_t c = 0; c < nc; ++c) {
      std::memcpy(&wrec[8 * c], &geo_dev[4 * c], 16);
      std::memcpy(&wrec[8 * c + 4], &h.topo[4 * c], 16);
    }
    // The learned criterion's features that depend on the cell only, in FP32
    // from the FP32 images with the feature definitions' own expressions:
    // log10(M/M_tot)/3, |Q|_F/(M l^2), extents/l (3), log2(1 + depth)/log2(22),
    // |com - boundary centre|/l.  And the inverse permutation for direct sums.
    std::vector<float> fcell((size_t)nc * 8);
    const float mtot = h.mp[3];
    for (int64_t c = 0; c < nc; ++c) {
      float* o = &fcell[8 * c];
      const float* m = &h.mp[12 * c];
      const float* gc = &h.geo[4 * c];
      const float l = gc[3], M = m[3];
      const float qn = std::sqrt((m[4] * m[4] + m[5] * m[5] + m[6] * m[6]) +
                                 2.0f * (m[7] * m[7] + m[8] * m[8] + m[9] * m[9]));
      float s2 = 0.0f;
      for (int k = 0; k < 3; ++k) {
        const float d = m[k] - gc[k];
        s2 += d * d;
      }
      o[0] = std::log10(M / mtot) / 3.0f;
      o[1] = qn / (M * l * l);
      for (int k = 0; k < 3; ++k) o[2 + k] = (float)(h.box[6 * c + 3 + k] - h.box[6 * c + k]) / l;
      o[5] = std::log2(1.0f + (float)h.depth[c]) / std::log2(22.0f);
      o[6] = std::sqrt(s2) / l;
      o[7] = 0.0f;
    }
    std::vector<int32_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) iperm[h.perm[i]] = (int32_t)i;
    if ((rc = upload(fcell, &dt.fcell)) || (rc = upload(iperm, &dt.iperm))) return rc;
    if ((rc = upload(h.part, &dt.part)) || (rc = upload(h.perm, &dt.perm)) ||
        (rc = upload(h.topo, &dt.topo)) || (rc = upload(geo_dev, &dt.geo)) ||
        (rc = upload(wrec, &dt.wrec)) ||
        (rc = upload(h.mp, &dt.mp)) || (rc = upload(h.ginfo, &dt.ginfo)) ||
        (rc = upload(h.gbox, &dt.gbox)) || (rc = upload(h.work, &dt.work)))
      return rc;
    return alloc_walk_buffers();
  }

  // Rebuilds the tree of device-resident positions and masses in place: the
  // previous tree's buffers, events and evaluation stream are reused.
  int rebuild_on_device(const float* pos, const float* mass, int64_t n, int n_leaf, int n_group) {
    if (!pool) {
      pool = std::make_unique<SeqPool>();
      build_pools = std::make_unique<BuildPools>();
    }
    pool->rewind();
    h = HostTree();
    dt = DevTree{};
    wb = WalkBufs{};
    darr = DeviceArrays{};
    d_diag_part = d_diag = nullptr;
    have_diag = counts_valid = false;
    slot_c = slot_l = 0;
    d_mlp = nullptr;
    learned = false;
    d_wrec_com = nullptr;
    com_theta = -1.0f;
    dev = false;
    std::string err;
    if (build_device_tree(pos, mass, true, n, n_leaf, n_group, h, dt, darr, *this, stream, err,
                          build_pools.get()) != 0)
      return fail(err.find("must be") != std::string::npos ? OCTGRAV_EINVAL : OCTGRAV_EHIP,
                  g_err.empty() ? err : g_err);
    host_partial = true;
    return alloc_walk_buffers();
  }

  // Walk and list buffers, scratch, events and the evaluation stream (after
  // the tree arrays are on the device, from either build).
  int alloc_walk_buffers() {
    const int64_t n = h.n, ng = h.n_groups(), nw = h.n_work();
    if (dt.nc >= (int64_t(1) << 29))  // the walks' queue entries hold cell id << 3
      return fail(OCTGRAV_EINVAL, "tree has " + std::to_string(dt.nc) +
                                      " cells; the walks address at most 2^29 - 1");
    int rc;
    void* p;
    if ((rc = dalloc(&p, (size_t)ng * 16))) return rc;
    wb.cnt = (int32_t*)p;
    if ((rc = dalloc(&p, (size_t)(ng + 1) * 8))) return rc;
    wb.c_off = (int64_t*)p;
    if ((rc = dalloc(&p, (size_t)(ng + 1) * 8))) return rc;
    wb.l_off = (int64_t*)p;
    if ((rc = dalloc(&p, 8 * 8))) return rc;
    wb.tot = (int64_t*)p;
    if (!tot_host && hipHostMalloc((void**)&tot_host, 8 * 8) != hipSuccess) {
      (void)hipGetLastError();  // read_tot then copies into pageable memory
      tot_host = nullptr;
    }
    if ((rc = dalloc(&p, (size_t)scan_scratch_entries(ng) * 8))) return rc;
    wb.blk = (int64_t*)p;
    if ((rc = dalloc(&p, (size_t)std::max(ng, nw) * 4))) return rc;
    wb.ovf_list = (int32_t*)p;
    if ((rc = dalloc(&p, 4))) return rc;
    wb.ovf_count = (int32_t*)p;
    if ((rc = dalloc(&p, (size_t)std::max(ng, nw) * 4))) return rc;
    wb.ovf_list2 = (int32_t*)p;
    if ((rc = dalloc(&p, 4))) return rc;
    wb.ovf_count2 = (int32_t*)p;
    if ((rc = dalloc(&p, 9 * 64 * 4))) return rc;
    wb.wctr = (int32_t*)p;
    // Fallback frontier queues: a breadth-first FIFO never holds more than
    // two consecutive levels, hence at most twice the widest level; entries
    // of two words (the fused wave walk's child ranges).
    int64_t cap = 64;
    while (cap < 2 * h.max_level_cells + 64) cap <<= 1;
    wb.gq_cap = cap;
    wb.gq_waves = fallback_waves();
    // At most 4 GiB of queues.
    while (wb.gq_waves > 64 && (int64_t)wb.gq_waves * cap * 8 > (int64_t(1) << 32)) wb.gq_waves >>= 1;
    if ((rc = dalloc(&p, (size_t)wb.gq_waves * cap * 8))) return rc;
    wb.gq = (int32_t*)p;
    wb.lds_qcap = lds_queue_entries();
    wb.export_lists = 0;
    wb.cap_c = wb.cap_l = 0;
    wb.c_ids = wb.l_ids = nullptr;
    if ((rc = dalloc(&p, (size_t)diag_scratch_entries(n) * 8))) return rc;
    d_diag_part = (double*)p;
    if ((rc = dalloc(&p, 4 * 8))) return rc;
    d_diag = (double*)p;
    for (hipEvent_t& e : ev)
      if (!e && hipEventCreate(&e) != hipSuccess) return fail(OCTGRAV_EHIP, "hipEventCreate failed");
    for (hipEvent_t& e : bev)
      if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return fail(OCTGRAV_EHIP, "hipEventCreate failed");
    if (!eval_stream && hipStreamCreateWithFlags(&eval_stream, hipStreamNonBlocking) != hipSuccess)
      return fail(OCTGRAV_EHIP, "hipStreamCreate failed");
    gwork.clear();  // built on first use (group_work)
    dev = true;
    return OCTGRAV_OK;
  }

  // Makes the list buffers hold at least (need_c, need_l) entries.
  int reserve_lists(int64_t need_c, int64_t need_l) {
    int rc;
    void* p;
    if (need_c > wb.cap_c) {
      if (wb.c_ids) dfree(wb.c_ids);
      wb.c_ids = nullptr;
      wb.cap_c = 0;
      int64_t cap = need_c + need_c / 8 + 1024;
      if ((rc = dalloc(&p, (size_t)cap * 4))) return rc;
      wb.c_ids = (int32_t*)p;
      wb.cap_c = cap;
    }
    if (need_l > wb.cap_l) {
      if (wb.l_ids) dfree(wb.l_ids);
      wb.l_ids = nullptr;
      wb.cap_l = 0;
      int64_t cap = need_l + need_l / 8 + 1024;
      if ((rc = dalloc(&p, (size_t)cap * 4))) return rc;
      wb.l_ids = (int32_t*)p;
      wb.cap_l = cap;
    }
    return OCTGRAV_OK;
  }

  int read_tot(int64_t* tot8) {
    int64_t* dst = tot_host ? tot_host : tot8;  // page-locked when the handle has it
    if (hipMemcpyAsync(dst, wb.tot, 8 * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return fail(OCTGRAV_EHIP, std::string("device error: ") + hipGetErrorString(hipGetLastError()));
    if (dst != tot8) std::memcpy(tot8, dst, 8 * 8);
    return OCTGRAV_OK;
  }

  // Two-pass path, pipelined over batches of groups: on the handle's stream
  // each batch's count walk, offsets and write walk; on eval_stream its
  // evaluation, which waits only for that batch's lists.  Needs list buffers
  // sized by an earlier call; a group whose lists do not fit is skipped and
  // reported through the totals, and the caller redoes the call.
  // First work item of every group (and nw at [ng]), from the host's work
  // list, fetched from the device for a device-built tree.
  int group_work() {
    const int64_t ng = h.n_groups(), nw = h.n_work();
    if ((int64_t)gwork.size() == ng + 1) return OCTGRAV_OK;
    if ((int64_t)h.work.size() != 2 * nw) {
      h.work.resize((size_t)nw * 2);
      if (nw > 0 && hipMemcpy(h.work.data(), dt.work, (size_t)nw * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(OCTGRAV_EHIP, "work list copy failed");
    }
    gwork.assign(ng + 1, nw);
    for (int64_t w = nw - 1; w >= 0; --w) gwork[h.work[2 * w]] = w;
    return OCTGRAV_OK;
  }

  int two_pass_pipelined(float theta, float eps, bool plain, float* acc, float* pot) {
    if (int rc = group_work()) return rc;
    const int64_t ng = h.n_groups();
    const int nb = (int)std::min<int64_t>(kBatches, std::max<int64_t>(1, ng / 256));
    WalkBufs ws = wb;  // slotted lists: no offsets scan between the walk and the evaluation
    ws.slot_c = slot_c;
    ws.slot_l = slot_l;
    hipEventRecord(bev[kBatches], stream);
    hipStreamWaitEvent(eval_stream, bev[kBatches], 0);
    for (int b = 0; b < nb; ++b) {
      const int64_t g0 = ng * b / nb, g1 = ng * (b + 1) / nb;
      if (launch_walk(dt, ws, theta, 2, stream, g0, g1 - g0, b == 0))
        return fail(OCTGRAV_EHIP, "walk launch failed");
      hipEventRecord(bev[b], stream);
      hipStreamWaitEvent(eval_stream, bev[b], 0);
      if (launch_eval(dt, ws, eps, plain, acc, pot, eval_stream, gwork[g0], gwork[g1] - gwork[g0]))
        return fail(OCTGRAV_EHIP, "evaluation launch failed");
    }
    if (launch_totals(dt, ws, stream)) return fail(OCTGRAV_EHIP, "totals launch failed");
    hipEventRecord(bev[kBatches + 1], eval_stream);
    hipStreamWaitEvent(stream, bev[kBatches + 1], 0);
    return OCTGRAV_OK;
  }

  // Slot sizes for the next pipelined call from the longest lists of this
  // one (tot[6], tot[7]), with headroom; the buffers are grown to match.
  int size_slots(const int64_t* tot) {
    const int64_t ng = h.n_groups();
    slot_c = (tot[6] + tot[6] / 4 + 63) / 64 * 64 + 64;
    slot_l = (tot[7] + tot[7] / 4 + 63) / 64 * 64 + 64;
    return reserve_lists(std::max(tot[0], ng * slot_c), std::max(tot[1], ng * slot_l));
  }

  // Count walk + offsets, then sizes the lists (a host read-back only when
  // the current capacity might not suffice), then the write walk.
  int lists_on_device(float theta, bool timed) {
    if (timed) hipEventRecord(ev[0], stream);
    if (launch_walk(dt, wb, theta, 0, stream)) return fail(OCTGRAV_EHIP, "count walk launch failed");
    if (timed) hipEventRecord(ev[1], stream);
    if (launch_scan(dt, wb, stream)) return fail(OCTGRAV_EHIP, "offsets launch failed");
    if (timed) hipEventRecord(ev[2], stream);
    if (wb.cap_c == 0) {
      int64_t tot[8];
      if (int rc = read_tot(tot)) return rc;
      if (tot[5]) return fail(OCTGRAV_ECAPACITY, "fallback walk frontier overflow");
      if (int rc = reserve_lists(tot[0], tot[1])) return rc;
    }
    if (launch_walk(dt, wb, theta, 1, stream)) return fail(OCTGRAV_EHIP, "write walk launch failed");
    if (timed) hipEventRecord(ev[3], stream);
    return OCTGRAV_OK;
  }
};

extern "C" {

const char* octgrav_last_error(void) { return g_err.c_str(); }

octgrav_tree* octgrav_build_tree_ex(const float* pos, const float* mass, int64_t n, int32_t n_leaf,
                                    int32_t n_group, uint32_t flags) {
  g_err.clear();
  try {
    std::string err;
    if ((flags & OCTGRAV_BUILD_DEVICE) && (flags & OCTGRAV_BUILD_HOST_ONLY)) {
      fail(OCTGRAV_EINVAL, "OCTGRAV_BUILD_DEVICE and OCTGRAV_BUILD_HOST_ONLY exclude each other");
      return nullptr;
    }
    if (flags & OCTGRAV_BUILD_DEVICE) {
      if (!validate_inputs(pos, mass, n, n_leaf, n_group, err)) {
        fail(OCTGRAV_EINVAL, err);
        return nullptr;
      }
      octgrav_tree* t = new octgrav_tree;
      if (build_device_tree(pos, mass, false, n, n_leaf, n_group, t->h, t->dt, t->darr, *t,
                            t->stream, err) != 0) {
        std::string keep = g_err.empty() ? err : g_err;
        delete t;
        fail(OCTGRAV_EHIP, keep);
        return nullptr;
      }
      t->host_partial = true;
      if (t->alloc_walk_buffers() != OCTGRAV_OK) {
        std::string keep = g_err;
        delete t;
        g_err = keep;
        return nullptr;
      }
      return t;
    }
    octgrav_tree* t = new octgrav_tree;
    if (!build_host_tree(pos, mass, n, n_leaf, n_group, t->h, err)) {
      delete t;
      fail(OCTGRAV_EINVAL, err);
      return nullptr;
    }
    if (!(flags & OCTGRAV_BUILD_HOST_ONLY)) {
      if (t->to_device() != OCTGRAV_OK) {
        std::string keep = g_err;
        delete t;
        g_err = keep;
        return nullptr;
      }
    }
    return t;
  } catch (const std::bad_alloc&) {
    fail(OCTGRAV_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    fail(OCTGRAV_EHIP, e.what());
  }
  return nullptr;
}

octgrav_tree* octgrav_build_tree(const float* pos, const float* mass, int64_t n, int32_t n_leaf) {
  return octgrav_build_tree_ex(pos, mass, n, n_leaf, 64, 0);
}

void octgrav_free(octgrav_tree* t) { delete t; }

int octgrav_set_stream(octgrav_tree* t, void* hip_stream) {
  if (!t) return fail(OCTGRAV_EINVAL, "NULL handle");
  t->stream = (hipStream_t)hip_stream;
  return OCTGRAV_OK;
}

int octgrav_tree_stats(const octgrav_tree* t, octgrav_stats* s) {
  if (!t || !s) return fail(OCTGRAV_EINVAL, "NULL argument");
  const HostTree& h = t->h;
  int64_t leaves = h.n_leaves;
  if (leaves < 0) {
    leaves = 0;
    for (int64_t c = 0; c < h.n_cells(); ++c) leaves += h.topo[4 * c + 1] == 0;
  }
  s->n = h.n;
  s->n_cells = h.n_cells();
  s->n_leaves = leaves;
  s->n_groups = h.n_groups();
  s->max_depth = h.max_depth;
  s->max_level_cells = h.max_level_cells;
  s->n_work = h.n_work();
  s->n_leaf = h.n_leaf;
  s->n_group = h.n_group;
  return OCTGRAV_OK;
}

int octgrav_export_tree(const octgrav_tree* t, const octgrav_tree_view* v) {
  if (!t || !v) return fail(OCTGRAV_EINVAL, "NULL argument");
  // A device-built tree copies its arrays back on the first export.
  if (int rc = const_cast<octgrav_tree*>(t)->fetch_host_arrays()) return rc;
  const HostTree& h = t->h;
  auto cp = [](auto* dst, const auto& src) {
    if (dst) std::memcpy(dst, src.data(), src.size() * sizeof(src[0]));
  };
  cp(v->perm, h.perm);
  cp(v->topo, h.topo);
  cp(v->geo, h.geo);
  cp(v->mp, h.mp);
  cp(v->mp64, h.mp64);
  cp(v->box, h.box);
  cp(v->depth, h.depth);
  cp(v->groups, h.groups);
  if (v->cube) {
    for (int k = 0; k < 3; ++k) v->cube[k] = h.corner[k];
    v->cube[3] = h.side;
  }
  return OCTGRAV_OK;
}

enum class Path { TwoPass, FusedBlock, FusedWave };

// Path of a call: an explicit flag, else the fused wave walk, the fastest
// measured at every angle (ms, fused wave / fused block, at theta 0.3, 0.35,
// 0.4, 0.5: 2^20 Plummer 8.95 / 11.0, 6.19 / 7.60, 4.30 / 5.46, 2.59 / 3.19;
// 4M clumps 34.5 / 43.4, 23.5 / 30.0, 16.8 / 21.6, 10.2 / 12.6; the two-pass
// path trails both).  The wave walk's queue entries of up to eight children
// keep its 512-entry LDS frontiers from overflowing down to theta 0.3, so it
// runs 16 walks per CU where the block walk runs four.
static Path choose_path(uint32_t flags) {
  if (flags & OCTGRAV_TWO_PASS) return Path::TwoPass;
  if (flags & OCTGRAV_FUSED_BLOCK) return Path::FusedBlock;
  return Path::FusedWave;
}

static int launch_fused(const octgrav_tree* t, Path p, float theta, float eps, bool plain,
                        bool do_eval, float* acc, float* pot) {
  int rc = p == Path::FusedWave
               ? launch_walk_eval(t->dt, t->wb, theta, eps, plain, do_eval, acc, pot, t->stream)
               : launch_walk_eval_block(t->dt, t->wb, theta, eps, plain, do_eval, acc, pot, t->stream);
  return rc ? rc : launch_totals(t->dt, t->wb, t->stream);
}

// While alive, the handle's walks read the offset test's records at theta
// (the evaluation's arrays are unchanged).
struct ComRecords {
  octgrav_tree* t = nullptr;
  const float* saved = nullptr;
  int rc = OCTGRAV_OK;
  ComRecords(octgrav_tree* tt, bool on, float theta) {
    if (!on) return;
    if (!tt->d_wrec_com) {
      void* p = nullptr;
      if ((rc = tt->dalloc(&p, (size_t)tt->dt.nc * 32))) return;
      tt->d_wrec_com = (float*)p;
      tt->com_theta = -1.0f;
    }
    if (tt->com_theta != theta) {
      if (launch_com_records(tt->dt, theta, tt->d_wrec_com, tt->stream)) {
        rc = fail(OCTGRAV_EHIP, "offset-test record launch failed");
        return;
      }
      tt->com_theta = theta;
    }
    t = tt;
    saved = tt->dt.wrec;
    tt->dt.wrec = tt->d_wrec_com;
  }
  ~ComRecords() {
    if (t) t->dt.wrec = saved;
  }
};

// Argument rules of OCTGRAV_MAC_COM.
static int check_com(const octgrav_tree* t, uint32_t flags, float theta) {
  if (!(flags & OCTGRAV_MAC_COM)) return OCTGRAV_OK;
  if (t->learned) return fail(OCTGRAV_EINVAL, "the offset test and the learned criterion exclude each other");
  if (flags & (OCTGRAV_TWO_PASS | OCTGRAV_FUSED_BLOCK))
    return fail(OCTGRAV_EINVAL, "the offset test runs on the fused wave path only");
  if (!(theta <= 0.57f)) return fail(OCTGRAV_EINVAL, "the offset test takes theta in [0, 0.57]");
  return OCTGRAV_OK;
}

static int check_theta(const octgrav_tree* t, float theta) {
  if (!t) return fail(OCTGRAV_EINVAL, "NULL handle");
  if (!t->dev) return fail(OCTGRAV_EINVAL, "tree was built host-only");
  if (!(theta >= 0.0f && theta <= 1.0f)) return fail(OCTGRAV_EINVAL, "theta must be in [0, 1]");
  return OCTGRAV_OK;
}

int octgrav_forces_ex(octgrav_tree* t, float theta, float eps, float* acc, float* pot,
                      uint32_t flags) {
  g_err.clear();
  if (int rc = check_theta(t, theta)) return rc;
  if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(OCTGRAV_EINVAL, "eps must be finite and > 0");
  if (!acc) return fail(OCTGRAV_EINVAL, "acc must be non-NULL");
  try {
    const bool timed = flags & OCTGRAV_TIMED, plain = flags & OCTGRAV_PLAIN_SUM;
    t->counts_valid = false;
    t->have_diag = false;
    int64_t tot[8];
    if (t->learned && (flags & (OCTGRAV_TWO_PASS | OCTGRAV_FUSED_BLOCK)))
      return fail(OCTGRAV_EINVAL, "the learned criterion runs on the fused wave path only");
    if (int rc = check_com(t, flags, theta)) return rc;
    const bool com = flags & OCTGRAV_MAC_COM;
    const Path path = (t->learned || com) ? Path::FusedWave : choose_path(flags);
    ComRecords cr(t, com, theta);
    if (cr.rc) return cr.rc;
    for (int attempt = 0; attempt < 2; ++attempt) {
      if (timed) {
        for (int k = 0; k < 4; ++k) hipEventRecord(t->ev[k], t->stream);
      }
      if (path != Path::TwoPass) {
        // Fused walk + evaluation: no lists in memory, no host round trip.
        t->wb.export_lists = 0;
        if (launch_fused(t, path, theta, eps, plain, true, acc, pot))
          return fail(OCTGRAV_EHIP, "walk+evaluation launch failed");
      } else if (t->slot_c > 0 && attempt == 0) {
        if (int rc = t->two_pass_pipelined(theta, eps, plain, acc, pot)) return rc;
      } else {
        // First call on this handle (the count walk sizes the list buffers),
        // or a retry after the lists outgrew them.
        if (int rc = t->lists_on_device(theta, timed)) return rc;
        if (launch_eval(t->dt, t->wb, eps, plain, acc, pot, t->stream))
          return fail(OCTGRAV_EHIP, "evaluation launch failed");
      }
      if (timed) hipEventRecord(t->ev[4], t->stream);
      if (launch_diag(t->dt, acc, pot, t->d_diag_part, t->d_diag, t->stream))
        return fail(OCTGRAV_EHIP, "diagnostics launch failed");
      if (timed) hipEventRecord(t->ev[5], t->stream);
      if (int rc = t->read_tot(tot)) return rc;
      if (debug_trace()) {
        int32_t ovf[2] = {0, 0};  // work items redone by the second / last walk tier
        if (path != Path::TwoPass) {
          hipMemcpy(&ovf[0], t->wb.ovf_count, 4, hipMemcpyDeviceToHost);
          hipMemcpy(&ovf[1], t->wb.ovf_count2, 4, hipMemcpyDeviceToHost);
        }
        std::fprintf(stderr,
                     "octgrav: attempt %d path %d slots %lld/%lld cap %lld/%lld tot %lld %lld %lld "
                     "%lld %lld %lld %lld %lld overflow %d %d\n",
                     attempt, (int)path, (long long)t->slot_c, (long long)t->slot_l,
                     (long long)t->wb.cap_c, (long long)t->wb.cap_l, (long long)tot[0],
                     (long long)tot[1], (long long)tot[2], (long long)tot[3], (long long)tot[4],
                     (long long)tot[5], (long long)tot[6], (long long)tot[7], ovf[0], ovf[1]);
      }
      if (tot[5]) return fail(OCTGRAV_ECAPACITY, "fallback walk frontier overflow");
      if (path != Path::TwoPass) break;
      const bool slotted = t->slot_c > 0 && attempt == 0;
      const bool fits = slotted ? !tot[4] : (tot[0] <= t->wb.cap_c && tot[1] <= t->wb.cap_l);
      if (fits) {
        if (!slotted)
          if (int rc = t->size_slots(tot)) return rc;
        break;
      }
      if (attempt == 1) return fail(OCTGRAV_ECAPACITY, "list capacity still exceeded after retry");
      // Slotted lists outgrew their slots: redo exactly (count walk, offsets,
      // write walk), which also resizes the slots for later calls.
      if (int rc = t->reserve_lists(tot[0], tot[1])) return rc;
      t->slot_c = t->slot_l = 0;
    }
    t->counts_valid = true;
    t->have_diag = true;
    if (timed) {
      float ms;
      for (int k = 0; k < 5; ++k) {
        hipEventElapsedTime(&ms, t->ev[k], t->ev[k + 1]);
        t->timings[k] = ms;
      }
      hipEventElapsedTime(&ms, t->ev[0], t->ev[5]);
      t->timings[5] = ms;
    }
    return OCTGRAV_OK;
  } catch (const std::exception& e) {
    return fail(OCTGRAV_EHIP, e.what());
  }
}

int octgrav_forces(octgrav_tree* t, float theta, float eps, float* acc, float* pot) {
  return octgrav_forces_ex(t, theta, eps, acc, pot, 0);
}

// Test hook: OCTGRAV_NOALLOC_LIMIT=<bytes> lowers the usable part of the
// no-allocation scratch (to reach the size check with small trees).
static size_t noalloc_limit() {
  size_t cap = noalloc_scratch_bytes();
  if (const char* v = std::getenv("OCTGRAV_NOALLOC_LIMIT")) {
    const long long x = std::atoll(v);
    if (x > 0 && (size_t)x < cap) cap = (size_t)x;
  }
  return cap;
}

int octgrav_forces_noalloc(octgrav_tree* t, float theta, float eps, float* acc, float* pot) {
  g_err.clear();
  if (int rc = check_theta(t, theta)) return rc;
  if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(OCTGRAV_EINVAL, "eps must be finite and > 0");
  if (!acc) return fail(OCTGRAV_EINVAL, "acc must be non-NULL");
  try {
    void* base = nullptr;
    std::string err;
    if (noalloc_scratch(&base, err)) return fail(OCTGRAV_EHIP, err);
    // Carve the per-call scratch of the fused walk + evaluation (and of the
    // diagnostics' partial sums) out of the array: fixed parts first, then as
    // many fallback frontier queues as fit (at least one).
    const int64_t ng = t->h.n_groups(), nw = t->h.n_work();
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t at = off;
      off += (bytes + 255) / 256 * 256;
      return (unsigned char*)base + at;
    };
    WalkBufs b = t->wb;
    b.tot = (int64_t*)take(8 * 8);
    b.wctr = (int32_t*)take(9 * 64 * 4);
    b.ovf_count = (int32_t*)take(4);
    b.ovf_count2 = (int32_t*)take(4);
    b.c_off = (int64_t*)take(8);  // only [0] is written without list export
    b.l_off = (int64_t*)take(8);
    b.cnt = (int32_t*)take((size_t)ng * 16);
    b.ovf_list = (int32_t*)take((size_t)std::max(ng, nw) * 4);
    b.ovf_list2 = (int32_t*)take((size_t)std::max(ng, nw) * 4);
    double* part = (double*)take((size_t)diag_scratch_entries(t->h.n) * 8);
    const size_t limit = noalloc_limit(), qbytes = (size_t)t->wb.gq_cap * 8;
    if (off + qbytes > limit)
      return fail(OCTGRAV_EINVAL, "tree needs " + std::to_string(off + qbytes) +
                                      " bytes of scratch; octgrav_forces_noalloc has " +
                                      std::to_string(limit));
    b.gq = (int32_t*)take(0);
    b.gq_waves = (int32_t)std::min<size_t>((size_t)t->wb.gq_waves, (limit - off) / qbytes);
    b.export_lists = 0;
    b.tr_off = nullptr;
    b.tr_c = nullptr;
    b.tr_s = nullptr;
    t->counts_valid = false;
    t->have_diag = false;
    const Path path = t->learned ? Path::FusedWave : choose_path(0);
    const int rc = path == Path::FusedWave
                       ? launch_walk_eval(t->dt, b, theta, eps, false, true, acc, pot, t->stream)
                       : launch_walk_eval_block(t->dt, b, theta, eps, false, true, acc, pot, t->stream);
    if (rc || launch_totals(t->dt, b, t->stream) || launch_diag(t->dt, acc, pot, part, t->d_diag, t->stream))
      return fail(OCTGRAV_EHIP, "walk+evaluation launch failed");
    // The call's totals and per-group records become the handle's, as after
    // octgrav_forces (last_counts, mac_stats read them there).
    if (hipMemcpyAsync(t->wb.tot, b.tot, 8 * 8, hipMemcpyDeviceToDevice, t->stream) != hipSuccess ||
        hipMemcpyAsync(t->wb.cnt, b.cnt, (size_t)ng * 16, hipMemcpyDeviceToDevice, t->stream) != hipSuccess)
      return fail(OCTGRAV_EHIP, "record copy failed");
    int64_t tot[8];
    if (int rc2 = t->read_tot(tot)) return rc2;
    if (tot[5]) return fail(OCTGRAV_ECAPACITY, "fallback walk frontier overflow");
    t->counts_valid = true;
    t->have_diag = true;
    return OCTGRAV_OK;
  } catch (const std::exception& e) {
    return fail(OCTGRAV_EHIP, e.what());
  }
}

// Count walk, offsets and write walk of the path the flags select: the lists
// of every group at theta end on the device (wb.c_off, wb.l_off, wb.c_ids,
// wb.l_ids); *n_c, *n_l = entries.
static int lists_to_device(octgrav_tree* t, float theta, uint32_t flags, int64_t* n_c,
                           int64_t* n_l) {
  t->counts_valid = false;
  int64_t tot[8];
  if (t->learned && (flags & (OCTGRAV_TWO_PASS | OCTGRAV_FUSED_BLOCK)))
    return fail(OCTGRAV_EINVAL, "the learned criterion runs on the fused wave path only");
  if (int rc = check_com(t, flags, theta)) return rc;
  const bool com = flags & OCTGRAV_MAC_COM;
  ComRecords cr(t, com, theta);
  if (cr.rc) return cr.rc;
  // Count walk and offsets give the sizes; the buffers are made to fit.
  // (The learned criterion and the offset test count with the fused walk.)
  t->wb.export_lists = 0;
  const bool fused_count = t->learned || com;
  if (fused_count ? launch_fused(t, Path::FusedWave, theta, 1.0f, false, false, nullptr, nullptr) != 0
                  : launch_walk(t->dt, t->wb, theta, 0, t->stream) != 0)
    return fail(OCTGRAV_EHIP, "count walk launch failed");
  if (launch_scan(t->dt, t->wb, t->stream)) return fail(OCTGRAV_EHIP, "offsets launch failed");
  if (int rc = t->read_tot(tot)) return rc;
  if (tot[5]) return fail(OCTGRAV_ECAPACITY, "fallback walk frontier overflow");
  if (int rc = t->reserve_lists(tot[0], tot[1])) return rc;
  const Path path = fused_count ? Path::FusedWave : choose_path(flags);
  if (path == Path::TwoPass) {
    if (launch_walk(t->dt, t->wb, theta, 1, t->stream)) return fail(OCTGRAV_EHIP, "write walk launch failed");
  } else {
    t->wb.export_lists = 1;
    int rc = launch_fused(t, path, theta, 1.0f, false, false, nullptr, nullptr);
    t->wb.export_lists = 0;
    if (rc) return fail(OCTGRAV_EHIP, "walk (export) launch failed");
  }
  int64_t tot2[8];
  if (int rc = t->read_tot(tot2)) return rc;
  if (tot2[5]) return fail(OCTGRAV_ECAPACITY, "fallback walk frontier overflow");
  if (tot2[0] != tot[0] || tot2[1] != tot[1])
    return fail(OCTGRAV_ECAPACITY, "walk list sizes disagree with the count walk");
  t->counts_valid = true;
  *n_c = tot[0];
  *n_l = tot[1];
  return OCTGRAV_OK;
}

// A selection of group indices: n_sel >= 0 entries, each in [0, n_groups).
static int check_selection(const octgrav_tree* t, const int32_t* groups, int64_t n_sel) {
  if (n_sel < 0) return fail(OCTGRAV_EINVAL, "n_sel must be >= 0");
  if (n_sel > 0 && !groups) return fail(OCTGRAV_EINVAL, "groups must be non-NULL when n_sel > 0");
  const int64_t ng = t->h.n_groups();
  for (int64_t k = 0; k < n_sel; ++k)
    if (groups[k] < 0 || groups[k] >= ng)
      return fail(OCTGRAV_EINVAL, "group index " + std::to_string(groups[k]) + " outside [0, " +
                                      std::to_string(ng) + ")");
  return OCTGRAV_OK;
}

int octgrav_lists_ex(octgrav_tree* t, float theta, uint32_t flags, int64_t* c_off, int32_t* c_ids,
                     int64_t* l_off, int32_t* l_ids, int64_t* n_c, int64_t* n_l) {
  g_err.clear();
  if (int rc = check_theta(t, theta)) return rc;
  if (!n_c || !n_l) return fail(OCTGRAV_EINVAL, "n_c and n_l must be non-NULL");
  const bool want = c_off || c_ids || l_off || l_ids;
  if (want && !(c_off && c_ids && l_off && l_ids))
    return fail(OCTGRAV_EINVAL, "give all four list arrays or none");
  try {
    int64_t tc = 0, tl = 0;
    if (int rc = lists_to_device(t, theta, flags, &tc, &tl)) return rc;
    *n_c = tc;
    *n_l = tl;
    if (want) {
      const int64_t ng = t->h.n_groups();
      if (hipMemcpy(c_off, t->wb.c_off, (ng + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(l_off, t->wb.l_off, (ng + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          (tc && hipMemcpy(c_ids, t->wb.c_ids, tc * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
          (tl && hipMemcpy(l_ids, t->wb.l_ids, tl * 4, hipMemcpyDeviceToHost) != hipSuccess))
        return fail(OCTGRAV_EHIP, "list copy-back failed");
    }
    return OCTGRAV_OK;
  } catch (const std::exception& e) {
    return fail(OCTGRAV_EHIP, e.what());
  }
}

int octgrav_lists_select(octgrav_tree* t, float theta, uint32_t flags, const int32_t* groups,
                         int64_t n_sel, int64_t* c_off, int32_t* c_ids, int64_t* l_off,
                         int32_t* l_ids, int64_t* n_c, int64_t* n_l) {
  g_err.clear();
  if (int rc = check_theta(t, theta)) return rc;
  if (!n_c || !n_l) return fail(OCTGRAV_EINVAL, "n_c and n_l must be non-NULL");
  if (int rc = check_selection(t, groups, n_sel)) return rc;
  const bool want = c_off || c_ids || l_off || l_ids;
  if (want && !(c_off && c_ids && l_off && l_ids))
    return fail(OCTGRAV_EINVAL, "give all four list arrays or none");
  try {
    int64_t tc = 0, tl = 0;
    if (int rc = lists_to_device(t, theta, flags, &tc, &tl)) return rc;
    const int64_t ng = t->h.n_groups();
    std::vector<int64_t> co(ng + 1), lo(ng + 1);
    if (hipMemcpy(co.data(), t->wb.c_off, (ng + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(lo.data(), t->wb.l_off, (ng + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(OCTGRAV_EHIP, "offset copy-back failed");
    int64_t sc = 0, sl = 0;
    for (int64_t k = 0; k < n_sel; ++k) {
      const int32_t g = groups[k];
      if (want) {
        c_off[k] = sc;
        l_off[k] = sl;
        const int64_t kc = co[g + 1] - co[g], kl = lo[g + 1] - lo[g];
        if ((kc && hipMemcpy(c_ids + sc, t->wb.c_ids + co[g], kc * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
            (kl && hipMemcpy(l_ids + sl, t->wb.l_ids + lo[g], kl * 4, hipMemcpyDeviceToHost) != hipSuccess))
          return fail(OCTGRAV_EHIP, "list copy-back failed");
      }
      sc += co[g + 1] - co[g];
      sl += lo[g + 1] - lo[g];
    }
    if (want) {
      c_off[n_sel] = sc;
      l_off[n_sel] = sl;
    }
    *n_c = sc;
    *n_l = sl;
    return OCTGRAV_OK;
  } catch (const std::exception& e) {
    return fail(OCTGRAV_EHIP, e.what());
  }
}

int octgrav_lists(octgrav_tree* t, float theta, int64_t* c_off, int32_t* c_ids, int64_t* l_off,
                  int32_t* l_ids, int64_t* n_c, int64_t* n_l) {
  return octgrav_lists_ex(t, theta, 0, c_off, c_ids, l_off, l_ids, n_c, n_l);
}

int octgrav_diagnostics(octgrav_tree* t, double mom[3], double* w) {
  if (!t || !mom || !w) return fail(OCTGRAV_EINVAL, "NULL argument");
  if (!t->have_diag) return fail(OCTGRAV_EINVAL, "no completed forces call on this handle");
  double out[4];
  if (hipMemcpy(out, t->d_diag, 32, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(OCTGRAV_EHIP, "diagnostics copy-back failed");
  for (int k = 0; k < 3; ++k) mom[k] = out[k];
  *w = out[3];
  return OCTGRAV_OK;
}

int octgrav_last_counts(octgrav_tree* t, int64_t out[4]) {
  if (!t || !out) return fail(OCTGRAV_EINVAL, "NULL argument");
  if (!t->counts_valid) return fail(OCTGRAV_EINVAL, "no completed forces/lists call");
  int64_t tot[8];
  if (int rc = t->read_tot(tot)) return rc;
  for (int k = 0; k < 4; ++k) out[k] = tot[k];
  return OCTGRAV_OK;
}

int octgrav_group_counts(octgrav_tree* t, int32_t* out) {
  if (!t || !out) return fail(OCTGRAV_EINVAL, "NULL argument");
  if (!t->counts_valid) return fail(OCTGRAV_EINVAL, "no completed forces/lists call");
  const int64_t ng = t->h.n_groups();
  if (ng > 0 && hipMemcpy(out, t->wb.cnt, (size_t)ng * 16, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(OCTGRAV_EHIP, "group counts copy failed");
  return OCTGRAV_OK;
}

int octgrav_direct(octgrav_tree* t, float eps, const int32_t* targets, int64_t nt, float* acc,
                   float* pot) {
  g_err.clear();
  if (!t) return fail(OCTGRAV_EINVAL, "NULL handle");
  if (!t->dev) return fail(OCTGRAV_EINVAL, "tree was built host-only");
  if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(OCTGRAV_EINVAL, "eps must be finite and > 0");
  if (!acc) return fail(OCTGRAV_EINVAL, "acc must be non-NULL");
  if (!targets) nt = t->h.n;
  if (nt < 0) return fail(OCTGRAV_EINVAL, "nt must be >= 0");
  if (targets && nt > 0) {  // indices are checked on the host before any kernel reads them
    std::vector<int32_t> tg(nt);
    if (hipMemcpy(tg.data(), targets, nt * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(OCTGRAV_EINVAL, "targets is not readable device memory");
    for (int32_t v : tg)
      if (v < 0 || v >= t->h.n) return fail(OCTGRAV_EINVAL, "target index out of range");
  }
  if (launch_direct(t->dt, targets, nt, eps, acc, pot, t->stream))
    return fail(OCTGRAV_EHIP, "direct-sum launch failed");
  if (hipStreamSynchronize(t->stream) != hipSuccess)
    return fail(OCTGRAV_EHIP, std::string("device error: ") + hipGetErrorString(hipGetLastError()));
  return OCTGRAV_OK;
}

int octgrav_mac_collect(octgrav_tree* t, float theta_lo, float theta_hi, float eps,
                        const float* acc_direct, int32_t stride, float* feat, float* label,
                        int32_t* group_out, int32_t* cell_out, int64_t cap, int64_t* n_out) {
  g_err.clear();
  if (int rc = check_theta(t, theta_lo)) return rc;
  if (!(theta_hi > theta_lo && theta_hi <= 1.0f)) return fail(OCTGRAV_EINVAL, "need theta_lo < theta_hi <= 1");
  if (!(eps > 0.0f)) return fail(OCTGRAV_EINVAL, "eps must be > 0");
  if (!acc_direct || !feat || !label || !n_out || stride < 1 || cap < 0)
    return fail(OCTGRAV_EINVAL, "bad collect arguments");
  try {
    // Band lists of every group (count walk, offsets, write walk in band mode).
    // They replace the handle's lists: the counts of the last forces call are gone.
    t->counts_valid = false;
    WalkBufs saved = t->wb;
    t->wb.band = 1;
    t->wb.band_hi2 = theta_hi * theta_hi;
    int64_t tot[8];
    int rc = 0;
    if (launch_walk(t->dt, t->wb, theta_lo, 0, t->stream) || launch_scan(t->dt, t->wb, t->stream))
      rc = fail(OCTGRAV_EHIP, "band walk launch failed");
    if (!rc) rc = t->read_tot(tot);
    if (!rc && tot[5]) rc = fail(OCTGRAV_ECAPACITY, "fallback walk frontier overflow");
    if (!rc) rc = t->reserve_lists(tot[0], 1);
    if (!rc) {
      WalkBufs b = t->wb;  // reserve_lists may have moved the buffers
      b.band = 1;
      b.band_hi2 = theta_hi * theta_hi;
      if (launch_walk(t->dt, b, theta_lo, 1, t->stream)) rc = fail(OCTGRAV_EHIP, "band walk launch failed");
    }
    const int64_t ng = t->h.n_groups();
    std::vector<int64_t> c_off(ng + 1);
    if (!rc && hipMemcpy(c_off.data(), t->wb.c_off, (ng + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess)
      rc = fail(OCTGRAV_EHIP, "offsets copy-back failed");
    t->wb.band = saved.band;
    t->wb.band_hi2 = saved.band_hi2;
    if (rc) return rc;
    // Sampled groups while their pairs fit.
    std::vector<int32_t> gs;
    std::vector<int64_t> off{0};
    for (int64_t g = 0; g < ng; g += stride) {
      const int64_t k = c_off[g + 1] - c_off[g];
      if (off.back() + k > cap) break;
      gs.push_back((int32_t)g);
      off.push_back(off.back() + k);
    }
    const int64_t np = off.back();
    *n_out = np;
    if (np == 0) return OCTGRAV_OK;
    void *dg = nullptr, *doff = nullptr;
    if ((rc = t->dalloc(&dg, gs.size() * 4)) || (rc = t->dalloc(&doff, off.size() * 8))) {
      t->dfree(dg);
      return rc;
    }
    if (hipMemcpy(dg, gs.data(), gs.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(doff, off.data(), off.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      t->dfree(dg);
      t->dfree(doff);
      return fail(OCTGRAV_EHIP, "sample upload failed");
    }
    rc = launch_mac_labels(t->dt, t->wb, (const int32_t*)dg, (int64_t)gs.size(), (const int64_t*)doff,
                           acc_direct, eps, feat, label, group_out, cell_out, np, t->stream);
    if (!rc && hipStreamSynchronize(t->stream) != hipSuccess) rc = -1;
    t->dfree(dg);
    t->dfree(doff);
    if (rc) return fail(OCTGRAV_EHIP, "label kernel failed");
    return OCTGRAV_OK;
  } catch (const std::exception& e) {
    return fail(OCTGRAV_EHIP, e.what());
  }
}

int octgrav_set_mac(octgrav_tree* t, const octgrav_mlp* m, float theta_lo, float theta_hi,
                    float tau_pair, float budget) {
  g_err.clear();
  if (!t) return fail(OCTGRAV_EINVAL, "NULL handle");
  if (!t->dev) return fail(OCTGRAV_EINVAL, "tree was built host-only");
  if (!m) {
    t->learned = false;
    t->wb.mlp = nullptr;
    return OCTGRAV_OK;
  }
  if (!(theta_lo > 0.0f && theta_lo < theta_hi && theta_hi <= 1.0f))
    return fail(OCTGRAV_EINVAL, "need 0 < theta_lo < theta_hi <= 1");
  if (!(tau_pair >= 0.0f) || std::isnan(budget)) return fail(OCTGRAV_EINVAL, "need tau_pair >= 0 and a budget");
  if (!t->d_mlp)
    if (int rc = t->dalloc(&t->d_mlp, kPkBytes)) return rc;
  if (hipMemcpy(t->d_mlp, m->pk, kPkBytes, hipMemcpyDeviceToDevice) != hipSuccess)
    return fail(OCTGRAV_EHIP, "network copy failed");
  t->learned = true;
  t->wb.mlp = (const uint8_t*)t->d_mlp;
  t->wb.mac_lo2 = theta_lo * theta_lo;
  t->wb.mac_hi2 = theta_hi * theta_hi;
  // log10 tau_pair: the FP64 logarithm of the FP32 value, rounded once to FP32
  // (reproducible anywhere; a float log10 may differ by an ulp between libraries)
  t->wb.mac_ltau = tau_pair > 0.0f ? (float)std::log10((double)tau_pair) : -INFINITY;
  t->wb.mac_budget = (double)budget;
  return OCTGRAV_OK;
}

// Per-group learned-walk records of the last fused call: band candidates
// visited and fall-back flags (host copies of cnt[].w).
static int read_band_counts(octgrav_tree* t, std::vector<int32_t>& w) {
  const int64_t ng = t->h.n_groups();
  std::vector<int32_t> cnt(4 * ng);
  if (hipMemcpy(cnt.data(), t->wb.cnt, ng * 16, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(OCTGRAV_EHIP, "count copy-back failed");
  w.resize(ng);
  for (int64_t g = 0; g < ng; ++g) w[g] = cnt[4 * g + 3];
  return OCTGRAV_OK;
}

int octgrav_mac_stats(octgrav_tree* t, int64_t out[2]) {
  g_err.clear();
  if (!t || !out) return fail(OCTGRAV_EINVAL, "NULL argument");
  if (!t->learned || !t->counts_valid)
    return fail(OCTGRAV_EINVAL, "no completed call with the learned criterion");
  std::vector<int32_t> w;
  if (int rc = read_band_counts(t, w)) return rc;
  out[0] = out[1] = 0;
  for (int32_t v : w) {
    out[0] += v >> 1;
    out[1] += v & 1;
  }
  return OCTGRAV_OK;
}

// Decision trace of the learned walks of the selected groups (sel == NULL:
// every group, in order).  The walk itself always covers every group; the
// selection only chooses what is copied back.
static int mac_trace_impl(octgrav_tree* t, float theta, const int32_t* sel, int64_t n_sel,
                          int64_t* off, int32_t* cells, float* scores, int64_t cap,
                          int64_t* n_out, int32_t* fell_back) {
  if (int rc = check_theta(t, theta)) return rc;
  if (!t->learned) return fail(OCTGRAV_EINVAL, "the learned criterion is not set");
  if (!off || !n_out || !fell_back) return fail(OCTGRAV_EINVAL, "off, n_out and fell_back must be non-NULL");
  try {
    t->counts_valid = false;
    const int64_t ng = t->h.n_groups();
    if (!sel) n_sel = ng;
    t->wb.export_lists = 0;
    if (launch_fused(t, Path::FusedWave, theta, 1.0f, false, false, nullptr, nullptr))
      return fail(OCTGRAV_EHIP, "walk launch failed");
    int64_t tot[8];
    if (int rc = t->read_tot(tot)) return rc;
    if (tot[5]) return fail(OCTGRAV_ECAPACITY, "fallback walk frontier overflow");
    std::vector<int32_t> w;
    if (int rc = read_band_counts(t, w)) return rc;
    std::vector<int64_t> full(ng + 1);
    full[0] = 0;
    for (int64_t g = 0; g < ng; ++g) full[g + 1] = full[g] + (w[g] >> 1);
    off[0] = 0;
    for (int64_t k = 0; k < n_sel; ++k) {
      const int64_t g = sel ? sel[k] : k;
      off[k + 1] = off[k] + (w[g] >> 1);
      fell_back[k] = w[g] & 1;
    }
    *n_out = off[n_sel];
    t->counts_valid = true;
    if (!cells || !scores) return OCTGRAV_OK;
    if (cap < off[n_sel]) return fail(OCTGRAV_EINVAL, "trace arrays too small");
    const int64_t nt = full[ng];
    void *d_off = nullptr, *d_c = nullptr, *d_s = nullptr;
    int rc = OCTGRAV_OK;
    if ((rc = t->dalloc(&d_off, (ng + 1) * 8)) || (rc = t->dalloc(&d_c, std::max<int64_t>(nt, 1) * 4)) ||
        (rc = t->dalloc(&d_s, std::max<int64_t>(nt, 1) * 4))) {
      t->dfree(d_off);
      t->dfree(d_c);
      return rc;
    }
    if (hipMemcpy(d_off, full.data(), (ng + 1) * 8, hipMemcpyHostToDevice) != hipSuccess) {
      t->dfree(d_off);
      t->dfree(d_c);
      t->dfree(d_s);
      return fail(OCTGRAV_EHIP, "trace offsets upload failed");
    }
    WalkBufs saved = t->wb;
    t->wb.tr_off = (const int64_t*)d_off;
    t->wb.tr_c = (int32_t*)d_c;
    t->wb.tr_s = (float*)d_s;
    if (launch_fused(t, Path::FusedWave, theta, 1.0f, false, false, nullptr, nullptr))
      rc = fail(OCTGRAV_EHIP, "walk launch failed");
    t->wb.tr_off = saved.tr_off;
    t->wb.tr_c = saved.tr_c;
    t->wb.tr_s = saved.tr_s;
    if (!rc && !sel && nt &&
        (hipMemcpy(cells, d_c, nt * 4, hipMemcpyDeviceToHost) != hipSuccess ||
         hipMemcpy(scores, d_s, nt * 4, hipMemcpyDeviceToHost) != hipSuccess))
      rc = fail(OCTGRAV_EHIP, "trace copy-back failed");
    for (int64_t k = 0; !rc && sel && k < n_sel; ++k) {
      const int64_t g = sel[k], len = full[g + 1] - full[g];
      if (len && (hipMemcpy(cells + off[k], (int32_t*)d_c + full[g], len * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                  hipMemcpy(scores + off[k], (float*)d_s + full[g], len * 4, hipMemcpyDeviceToHost) != hipSuccess))
        rc = fail(OCTGRAV_EHIP, "trace copy-back failed");
    }
    t->dfree(d_off);
    t->dfree(d_c);
    t->dfree(d_s);
    return rc;
  } catch (const std::exception& e) {
    return fail(OCTGRAV_EHIP, e.what());
  }
}

int octgrav_mac_trace(octgrav_tree* t, float theta, int64_t* off, int32_t* cells, float* scores,
                      int64_t cap, int64_t* n_out, int32_t* fell_back) {
  g_err.clear();
  return mac_trace_impl(t, theta, nullptr, 0, off, cells, scores, cap, n_out, fell_back);
}

int octgrav_mac_trace_select(octgrav_tree* t, float theta, const int32_t* groups, int64_t n_sel,
                             int64_t* off, int32_t* cells, float* scores, int64_t cap,
                             int64_t* n_out, int32_t* fell_back) {
  g_err.clear();
  if (!t) return fail(OCTGRAV_EINVAL, "NULL handle");
  if (int rc = check_selection(t, groups, n_sel)) return rc;
  if (n_sel == 0) {  // an empty selection: nothing to walk for
    if (int rc = check_theta(t, theta)) return rc;
    if (!t->learned) return fail(OCTGRAV_EINVAL, "the learned criterion is not set");
    if (!off || !n_out || !fell_back) return fail(OCTGRAV_EINVAL, "off, n_out and fell_back must be non-NULL");
    off[0] = 0;
    *n_out = 0;
    return OCTGRAV_OK;
  }
  return mac_trace_impl(t, theta, groups, n_sel, off, cells, scores, cap, n_out, fell_back);
}

// ------------------------------------------------------------------ network

octgrav_mlp* octgrav_mlp_create(const float* params) {
  g_err.clear();
  octgrav_mlp* m = new (std::nothrow) octgrav_mlp;
  if (!m) {
    fail(OCTGRAV_ENOMEM, "out of host memory");
    return nullptr;
  }
  std::vector<float> zero(kMlpParams, 0.0f);
  if (m->alloc(&m->P, kMlpParams * 4) || m->alloc(&m->mom1, kMlpParams * 4) ||
      m->alloc(&m->mom2, kMlpParams * 4) || m->alloc(&m->grad, kMlpParams * 4) ||
      m->alloc(&m->pk, kPkBytes) || m->alloc(&m->d_loss, 8) ||
      octgrav_mlp_set_params(m, params ? params : zero.data()) != OCTGRAV_OK) {
    octgrav_mlp_free(m);
    return nullptr;
  }
  return m;
}

void octgrav_mlp_free(octgrav_mlp* m) { delete m; }

int octgrav_mlp_set_stream(octgrav_mlp* m, void* hip_stream) {
  if (!m) return fail(OCTGRAV_EINVAL, "NULL handle");
  m->stream = (hipStream_t)hip_stream;
  return OCTGRAV_OK;
}

int octgrav_mlp_set_params(octgrav_mlp* m, const float* params) {
  g_err.clear();
  if (!m || !params) return fail(OCTGRAV_EINVAL, "NULL argument");
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(params[i])) return fail(OCTGRAV_EINVAL, "non-finite parameter");
  if (hipMemcpy(m->P, params, kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->mom1, 0, kMlpParams * 4) != hipSuccess ||
      hipMemset(m->mom2, 0, kMlpParams * 4) != hipSuccess)
    return fail(OCTGRAV_EHIP, "parameter upload failed");
  if (launch_mlp_pack((const float*)m->P, m->pk, m->stream) ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return fail(OCTGRAV_EHIP, "pack failed");
  return OCTGRAV_OK;
}

int octgrav_mlp_set_state(octgrav_mlp* m, const float* params, const float* mom1,
                          const float* mom2) {
  g_err.clear();
  if (!m || !params || !mom1 || !mom2) return fail(OCTGRAV_EINVAL, "NULL argument");
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(params[i]) || !std::isfinite(mom1[i]) || !std::isfinite(mom2[i]) ||
        mom2[i] < 0.0f)
      return fail(OCTGRAV_EINVAL, "non-finite parameter or moment, or negative second moment");
  if (hipMemcpy(m->P, params, kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->mom1, mom1, kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->mom2, mom2, kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail(OCTGRAV_EHIP, "state upload failed");
  if (launch_mlp_pack((const float*)m->P, m->pk, m->stream) ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return fail(OCTGRAV_EHIP, "pack failed");
  return OCTGRAV_OK;
}

int octgrav_mlp_get_moments(const octgrav_mlp* m, float* mom1, float* mom2) {
  g_err.clear();
  if (!m || !mom1 || !mom2) return fail(OCTGRAV_EINVAL, "NULL argument");
  if (hipStreamSynchronize(m->stream) != hipSuccess ||
      hipMemcpy(mom1, m->mom1, kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(mom2, m->mom2, kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(OCTGRAV_EHIP, "moment copy-back failed");
  return OCTGRAV_OK;
}

int octgrav_mlp_get_params(const octgrav_mlp* m, float* params) {
  g_err.clear();
  if (!m || !params) return fail(OCTGRAV_EINVAL, "NULL argument");
  if (hipStreamSynchronize(m->stream) != hipSuccess ||
      hipMemcpy(params, m->P, kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(OCTGRAV_EHIP, "parameter copy-back failed");
  return OCTGRAV_OK;
}

int octgrav_mlp_forward(octgrav_mlp* m, const float* x, int64_t b, float* y) {
  g_err.clear();
  if (!m) return fail(OCTGRAV_EINVAL, "NULL handle");
  if (b < 0 || (b > 0 && (!x || !y))) return fail(OCTGRAV_EINVAL, "bad batch arguments");
  if (launch_mlp_forward(m->pk, x, b, y, nullptr, nullptr, m->stream) ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return fail(OCTGRAV_EHIP, "forward failed");
  return OCTGRAV_OK;
}

int octgrav_mlp_loss_grad(octgrav_mlp* m, const float* x, const float* target, int64_t b,
                          float tau, double* loss, float* grad) {
  g_err.clear();
  if (!m || !loss) return fail(OCTGRAV_EINVAL, "NULL argument");
  if (b < 1 || !x || !target) return fail(OCTGRAV_EINVAL, "bad batch arguments");
  if (!(tau > 0.0f && tau < 1.0f)) return fail(OCTGRAV_EINVAL, "tau must be in (0, 1)");
  if (int rc = m->reserve(b)) return rc;
  if (launch_mlp_loss_grad(m->pk, x, target, b, tau, (float*)m->scratch, (float*)m->grad,
                           (double*)m->d_loss, m->stream) ||
      hipMemcpyAsync(loss, m->d_loss, 8, hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
      (grad && hipMemcpyAsync(grad, m->grad, kMlpParams * 4, hipMemcpyDeviceToHost, m->stream) !=
                   hipSuccess) ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return fail(OCTGRAV_EHIP, "loss/gradient failed");
  return OCTGRAV_OK;
}

int octgrav_mlp_adam(octgrav_mlp* m, float lr, float beta1, float beta2, float eps, int32_t step) {
  g_err.clear();
  if (!m) return fail(OCTGRAV_EINVAL, "NULL handle");
  if (step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f))
    return fail(OCTGRAV_EINVAL, "bad Adam arguments");
  const float c1 = (float)(1.0 - std::pow((double)beta1, step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, step));
  if (launch_mlp_adam((float*)m->P, (float*)m->mom1, (float*)m->mom2, (const float*)m->grad, lr,
                      beta1, beta2, eps, c1, c2, m->stream) ||
      launch_mlp_pack((const float*)m->P, m->pk, m->stream) ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return fail(OCTGRAV_EHIP, "Adam step failed");
  return OCTGRAV_OK;
}

// ------------------------------------------------------------------ integration

// A particle system on the device, integrated with kick-drift-kick leapfrog;
// the tree is rebuilt on the GPU from the drifted positions every step.
struct octgrav_sim {
  int64_t n = 0;
  int n_leaf = 16, n_group = 64;
  hipStream_t stream = nullptr;
  float *pos = nullptr, *vel = nullptr, *mass = nullptr, *acc = nullptr, *pot = nullptr;
  double *kpart = nullptr, *kout = nullptr;
  octgrav_tree* tree = nullptr;
  bool have_forces = false;
  // Set when a run fails after a step's first half-kick: velocities, positions
  // and accelerations no longer belong to one time, so the handle refuses
  // further runs, energies and states.
  bool broken = false;
  float theta = -1.0f, eps = -1.0f;
  double timings[3] = {0, 0, 0};  // last run: ms per step, of which tree build, forces

  ~octgrav_sim() {
    if (tree) octgrav_free(tree);
    for (void* p : {(void*)pos, (void*)vel, (void*)mass, (void*)acc, (void*)pot, (void*)kpart,
                    (void*)kout})
      if (p) hipFree(p);
  }

  // Tree of the current positions and the forces on them.
  // The handle is rebuilt in place, so its device buffers carry over from
  // one step to the next.
  int rebuild_and_force(double* t_build, double* t_force) {
    auto t0 = std::chrono::steady_clock::now();
    if (!tree) {
      tree = new (std::nothrow) octgrav_tree;
      if (!tree) return fail(OCTGRAV_ENOMEM, "out of host memory");
    }
    tree->stream = stream;
    have_forces = false;
    if (int rc = tree->rebuild_on_device(pos, mass, n, n_leaf, n_group)) return rc;
    auto t1 = std::chrono::steady_clock::now();
    if (int rc = octgrav_forces_ex(tree, theta, eps, acc, pot, 0)) return rc;
    auto t2 = std::chrono::steady_clock::now();
    *t_build += std::chrono::duration<double, std::milli>(t1 - t0).count();
    *t_force += std::chrono::duration<double, std::milli>(t2 - t1).count();
    have_forces = true;
    return OCTGRAV_OK;
  }
};

octgrav_sim* octgrav_sim_create(const float* pos, const float* vel, const float* mass, int64_t n,
                                int32_t n_leaf, int32_t n_group) {
  g_err.clear();
  std::string err;
  if (!vel) {
    fail(OCTGRAV_EINVAL, "vel must be non-NULL");
    return nullptr;
  }
  if (!validate_inputs(pos, mass, n, n_leaf, n_group, err)) {
    fail(OCTGRAV_EINVAL, err);
    return nullptr;
  }
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(vel[i])) {
      fail(OCTGRAV_EINVAL, "velocities must be finite");
      return nullptr;
    }
  octgrav_sim* s = new (std::nothrow) octgrav_sim;
  if (!s) {
    fail(OCTGRAV_ENOMEM, "out of host memory");
    return nullptr;
  }
  s->n = n;
  s->n_leaf = n_leaf;
  s->n_group = n_group;
  auto A = [&](void** p, size_t bytes) {
    if (alloc_fault() || hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return false;
    }
    return true;
  };
  if (!A((void**)&s->pos, n * 12) || !A((void**)&s->vel, n * 12) || !A((void**)&s->mass, n * 4) ||
      !A((void**)&s->acc, n * 12) || !A((void**)&s->pot, n * 4) ||
      !A((void**)&s->kpart, kinetic_scratch_entries() * 8) || !A((void**)&s->kout, 32)) {
    delete s;
    fail(OCTGRAV_ENOMEM, "device allocation failed");
    return nullptr;
  }
  if (hipMemcpy(s->pos, pos, n * 12, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->vel, vel, n * 12, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->mass, mass, n * 4, hipMemcpyHostToDevice) != hipSuccess) {
    delete s;
    fail(OCTGRAV_EHIP, "state upload failed");
    return nullptr;
  }
  return s;
}

void octgrav_sim_free(octgrav_sim* s) { delete s; }

int octgrav_sim_set_stream(octgrav_sim* s, void* hip_stream) {
  if (!s) return fail(OCTGRAV_EINVAL, "NULL handle");
  s->stream = (hipStream_t)hip_stream;
  if (s->tree) s->tree->stream = s->stream;
  return OCTGRAV_OK;
}

static int sim_broken() {
  return fail(OCTGRAV_EINVAL,
              "an earlier run failed in the middle of a step; the state is inconsistent");
}

int octgrav_sim_run(octgrav_sim* s, float theta, float eps, float dt, int32_t steps) {
  g_err.clear();
  if (!s) return fail(OCTGRAV_EINVAL, "NULL handle");
  if (s->broken) return sim_broken();
  if (!(theta >= 0.0f && theta <= 1.0f)) return fail(OCTGRAV_EINVAL, "theta must be in [0, 1]");
  if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(OCTGRAV_EINVAL, "eps must be finite and > 0");
  if (!std::isfinite(dt) || steps < 0) return fail(OCTGRAV_EINVAL, "bad dt or steps");
  try {
    double tb = 0, tf = 0;
    auto t0 = std::chrono::steady_clock::now();
    if (!s->have_forces || theta != s->theta || eps != s->eps) {
      s->theta = theta;
      s->eps = eps;
      if (int rc = s->rebuild_and_force(&tb, &tf)) return rc;
      tb = tf = 0;
      t0 = std::chrono::steady_clock::now();
    }
    for (int32_t k = 0; k < steps; ++k) {
      // From the first half-kick on, a failure leaves the step half done.
      s->broken = true;
      if (launch_kick(s->vel, s->acc, s->n, 0.5f * dt, s->stream) ||
          launch_drift(s->pos, s->vel, s->n, dt, s->stream))
        return fail(OCTGRAV_EHIP, "leapfrog launch failed");
      if (int rc = s->rebuild_and_force(&tb, &tf)) return rc;
      if (launch_kick(s->vel, s->acc, s->n, 0.5f * dt, s->stream))
        return fail(OCTGRAV_EHIP, "leapfrog launch failed");
      s->broken = false;
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) {
      s->broken = steps > 0;
      return fail(OCTGRAV_EHIP, "device error during integration");
    }
    if (steps > 0) {
      const double ms = std::chrono::duration<double, std::milli>(
                            std::chrono::steady_clock::now() - t0).count();
      s->timings[0] = ms / steps;
      s->timings[1] = tb / steps;
      s->timings[2] = tf / steps;
    }
    return OCTGRAV_OK;
  } catch (const std::exception& e) {
    return fail(OCTGRAV_EHIP, e.what());
  }
}

int octgrav_sim_energy(octgrav_sim* s, double out[6]) {
  g_err.clear();
  if (!s || !out) return fail(OCTGRAV_EINVAL, "NULL argument");
  if (s->broken) return sim_broken();
  if (!s->have_forces) return fail(OCTGRAV_EINVAL, "no forces yet: run at least once (steps may be 0)");
  double k4[4], mom[3], w;
  if (launch_kinetic(s->mass, s->vel, s->n, s->kpart, s->kout, s->stream) ||
      hipMemcpyAsync(k4, s->kout, 32, hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)
    return fail(OCTGRAV_EHIP, "kinetic energy failed");
  if (int rc = octgrav_diagnostics(s->tree, mom, &w)) return rc;
  out[0] = k4[0];
  out[1] = w;
  out[2] = k4[0] + w;
  out[3] = k4[1];
  out[4] = k4[2];
  out[5] = k4[3];
  return OCTGRAV_OK;
}

int octgrav_sim_state(const octgrav_sim* s, float* pos, float* vel, float* acc) {
  if (!s) return fail(OCTGRAV_EINVAL, "NULL handle");
  if (s->broken) return sim_broken();
  if (hipStreamSynchronize(s->stream) != hipSuccess ||
      (pos && hipMemcpy(pos, s->pos, s->n * 12, hipMemcpyDeviceToHost) != hipSuccess) ||
      (vel && hipMemcpy(vel, s->vel, s->n * 12, hipMemcpyDeviceToHost) != hipSuccess) ||
      (acc && s->have_forces && hipMemcpy(acc, s->acc, s->n * 12, hipMemcpyDeviceToHost) != hipSuccess))
    return fail(OCTGRAV_EHIP, "state copy-back failed");
  return OCTGRAV_OK;
}

int octgrav_sim_timings(const octgrav_sim* s, double out[3]) {
  if (!s || !out) return fail(OCTGRAV_EINVAL, "NULL argument");
  for (int k = 0; k < 3; ++k) out[k] = s->timings[k];
  return OCTGRAV_OK;
}

int octgrav_last_timings(octgrav_tree* t, double out[6]) {
  if (!t || !out) return fail(OCTGRAV_EINVAL, "NULL argument");
  for (int k = 0; k < 6; ++k) out[k] = t->timings[k];
  return OCTGRAV_OK;
}

}  // extern "C"
