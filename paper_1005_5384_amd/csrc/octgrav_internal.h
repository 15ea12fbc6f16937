// Internal declarations shared by the library's host and device sources.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace octgrav {

constexpr int kMaxDepth = 21;   // levels below the root cube (63-bit Morton keys)
constexpr int kChunk = 32;      // targets per evaluation work item

// Host tree (Sec. 2.1), FP64 geometry and moments, FP32 device images.
struct HostTree {
  int64_t n = 0;
  int n_leaf = 0, n_group = 0;
  double corner[3] = {0, 0, 0}, side = 1;   // root cube
  int max_depth = 0;
  int64_t max_level_cells = 0;
  int64_t n_leaves = -1;         // counted by the device build (-1: count from topo)
  std::vector<int32_t> perm;     // [n] sorted position -> input index
  std::vector<float> part;       // [n*4] sorted x, y, z, m
  std::vector<int32_t> topo;     // [nc*4] first_child, n_child, first, n
  std::vector<int32_t> depth;    // [nc]
  std::vector<double> box;       // [nc*6] tight box
  std::vector<double> mp64;      // [nc*10] M, com, Q (xx yy zz xy xz yz)
  std::vector<float> geo;        // [nc*4] f32 boundary centre, side
  std::vector<float> mp;         // [nc*12] f32 com, M | Qxx Qyy Qzz Qxy | Qxz Qyz 0 0
  std::vector<int32_t> groups;   // [ng] cell id
  std::vector<int32_t> ginfo;    // [ng*4] first, n, cell, 0
  std::vector<float> gbox;       // [ng*8] gmin xyz 0, gmax xyz 0
  std::vector<int32_t> work;     // [nw*2] group, first target offset within group
  // Counts of a device build whose depth / groups / work arrays stay on the
  // device until an export fetches them (-1: the vectors' sizes).
  int64_t nc_dev = -1, ng_dev = -1, nw_dev = -1;
  int64_t n_cells() const { return nc_dev >= 0 ? nc_dev : (int64_t)depth.size(); }
  int64_t n_groups() const { return ng_dev >= 0 ? ng_dev : (int64_t)groups.size(); }
  int64_t n_work() const { return nw_dev >= 0 ? nw_dev : (int64_t)work.size() / 2; }
};

// Builds the host tree; returns false with a message on bad input.
bool build_host_tree(const float* pos, const float* mass, int64_t n, int n_leaf, int n_group,
                     HostTree& out, std::string& err);
// Pieces shared by the host and device builds.
bool validate_inputs(const float* pos, const float* mass, int64_t n, int n_leaf, int n_group,
                     std::string& err);
void root_cube(const double lo[3], const double hi[3], double corner[3], double* side);

// ------------------------------------------------------------------ network
// Learned acceptance criterion: 12 -> 64 -> 64 -> 1 with ReLU.
constexpr int kMlpIn = 12, kMlpInPad = 16, kMlpH = 64;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;  // 5057
// FP32 parameter vector offsets: W1 [64 x 12] row-major, b1, W2 [64 x 64], b2, w3, b3.
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kMlpH * kMlpIn, kOffW2 = kOffB1 + kMlpH,
              kOffB2 = kOffW2 + kMlpH * kMlpH, kOffW3 = kOffB2 + kMlpH, kOffB3 = kOffW3 + kMlpH;

// Packed inference image (one device buffer), byte offsets.
constexpr int kPkW1 = 0;                              // BF16 [64][16]
constexpr int kPkW2 = kPkW1 + kMlpH * kMlpInPad * 2;  // BF16 [64][64]
constexpr int kPkB1 = kPkW2 + kMlpH * kMlpH * 2;      // FP32 [64]
constexpr int kPkB2 = kPkB1 + kMlpH * 4;              // FP32 [64]
constexpr int kPkW3 = kPkB2 + kMlpH * 4;              // BF16 [64]
constexpr int kPkB3 = kPkW3 + kMlpH * 2;              // FP32
constexpr int kPkBytes = kPkB3 + 256;

// ------------------------------------------------------------------ device
struct DevTree {
  const float* part;     // float4 [n]
  const int32_t* perm;   // [n]
  const int32_t* topo;   // int4 [nc]
  const float* geo;      // float4 [nc]  boundary; the side's sign bit marks leaves
  const float* wrec;     // float4 x2 [nc] walk record: boundary (as geo) | topo
  const float* fcell;    // float4 x2 [nc] learned-criterion features of the cell alone:
                         // f1, f2, f4, f5 | f6, f10, f11, 0 (see mac_features)
  const int32_t* iperm;  // [n] caller index -> sorted position
  const float* mp;       // float4 x3 [nc]
  const int32_t* ginfo;  // int4 [ng]
  const float* gbox;     // float4 x2 [ng]
  const int32_t* work;   // int2 [nw]
  int64_t n, nc, ng, nw;
};

struct WalkBufs {
  int32_t* cnt;        // int4 [ng]: |C|, |L|, n_src(L), frontier-overflow flag
  int64_t* c_off;      // [ng+1]
  int64_t* l_off;      // [ng+1]
  int32_t* c_ids;      // [cap_c]
  int32_t* l_ids;      // [cap_l]
  int64_t cap_c, cap_l;
  int64_t* tot;        // [8]: n_c, n_l, N_pc, N_pp, capacity-overflow, fallback-overflow
  int64_t* blk;        // scan scratch: 2 per scan block
  int32_t* ovf_list;   // [max(ng, nw)] groups / work items whose LDS frontier overflowed
  int32_t* ovf_count;  // [1]
  int32_t* ovf_list2;  // [max(ng, nw)] second-tier overflows (fused wave kernels)
  int32_t* ovf_count2; // [1]
  int32_t* wctr;       // [9 x 64]: work counters (stride 64) of persistent kernels:
                       // 8 per-XCD ranges, 1 overflow list
  int32_t* gq;         // global frontier queues for the fallback walk: 2 * gq_cap words each
  int64_t gq_cap;      // entries per queue (power of two)
  int32_t gq_waves;    // queues (waves) of the fallback walk
  int32_t lds_qcap;    // cap on the LDS frontier in candidates (power of two >= 64; test
                       // hook); the fused wave walk's entries of up to eight children use
                       // lds_qcap / 8 of them
  int32_t export_lists;  // fused walk: also write the lists at c_off / l_off
  // Slotted lists (walk mode 2, > 0): group g's lists start at g * slot_c /
  // g * slot_l and their lengths are cnt[g].x / .y; 0 = CSR offsets.
  int64_t slot_c, slot_l;
  // Band collection (band != 0): the "cell list" records the candidates the
  // walk's test opens and the test at band_hi2 (squared angle) does not.
  int32_t band;
  float band_hi2;
  // Learned acceptance criterion (fused wave walk; mlp == NULL: the theta
  // test).  Candidates the test at mac_lo2 accepts are accepted, those the
  // test at mac_hi2 opens are opened, the network decides the rest (accept
  // iff its output <= mac_ltau); a group whose accepted band candidates give
  // sqrt(sum 10^(2 y)) > mac_budget is walked again with the call's theta.
  // cnt[g].w = 2 * (band candidates visited) + (1 if the group fell back).
  const uint8_t* mlp;  // packed network image (mlp_device.h)
  float mac_lo2, mac_hi2, mac_ltau;
  double mac_budget;
  // Decision trace of the learned walks (test export; tr_s == NULL: off):
  // group g's band candidates at [tr_off[g], tr_off[g + 1]).
  const int64_t* tr_off;
  int32_t* tr_c;
  float* tr_s;
};

// Kernel launchers (device sources).  mode 0 = count, 1 = write at the
// offsets, 2 = count and write into per-group slots.  Ranges
// are [g0, g0 + ng) groups / [w0, w0 + nw) work items (ng, nw < 0: to the end).
int launch_walk(const DevTree& T, const WalkBufs& B, float theta, int mode, void* stream,
                int64_t g0 = 0, int64_t ng = -1, bool init = true);
int launch_scan(const DevTree& T, const WalkBufs& B, void* stream, int64_t g0 = 0, int64_t ng = -1);
// Interaction totals and longest lists from the per-group counts.
int launch_totals(const DevTree& T, const WalkBufs& B, void* stream, int64_t g0 = 0, int64_t ng = -1);
int launch_eval(const DevTree& T, const WalkBufs& B, float eps, bool plain, float* acc,
                float* pot, void* stream, int64_t w0 = 0, int64_t nw = -1);
int launch_walk_eval(const DevTree& T, const WalkBufs& B, float theta, float eps, bool plain,
                     bool do_eval, float* acc, float* pot, void* stream);
int launch_walk_eval_block(const DevTree& T, const WalkBufs& B, float theta, float eps, bool plain,
                           bool do_eval, float* acc, float* pot, void* stream);
// Walk records (nc x 32 B, the layout of DevTree::wrec) of the centre-of-mass
// offset opening test at theta: boundary (com, l + theta |com - cb|), topology.
int launch_com_records(const DevTree& T, float theta, float* out, void* stream);
// FP32 compensated direct sum for targets (caller indices, device array, or
// NULL = all); outputs in target order.
int launch_direct(const DevTree& T, const int32_t* targets, int64_t nt, float eps, float* acc,
                  float* pot, void* stream);
// Features (12, FP32) and labels of the band pairs of the listed groups
// (pair p of listed group s sits at out_off[s] + k); also each pair's ids.
int launch_mac_labels(const DevTree& T, const WalkBufs& B, const int32_t* groups, int64_t ngs,
                      const int64_t* out_off, const float* acc_direct, float eps, float* feat,
                      float* label, int32_t* gout, int32_t* cout, int64_t npairs, void* stream);
// Network of the learned criterion: pack FP32 parameters into the BF16
// inference image; batch forward (a1s / a2s: B x 64 pre-activations, may be
// NULL); loss + gradient of a batch (scratch arrays B x 64 / B); Adam step.
int launch_mlp_pack(const float* P, void* pk, void* stream);
int launch_mlp_forward(const void* pk, const float* x, int64_t B, float* y, float* a1s, float* a2s,
                       void* stream);
int launch_mlp_loss_grad(const void* pk, const float* x, const float* tgt, int64_t B, float tau,
                         float* scratch, float* grad, double* loss, void* stream);
int64_t mlp_train_scratch_floats(int64_t B);  // scratch of launch_mlp_loss_grad
int launch_mlp_adam(float* P, float* m, float* v, const float* g, float lr, float b1, float b2,
                    float eps, float c1, float c2, void* stream);
// Device tree build (same result as build_host_tree, computed on the GPU).
// The persistent arrays are allocated through DevAlloc (owned by the
// caller); DeviceArrays receives the FP64 boxes / moments, the unsigned
// boundary image, the depths and the group cells, which stay on the device.
// Fills h with the scalars and the counts (nc_dev, ng_dev, nw_dev); every
// array stays on the device.  A build with pools makes two host round trips
// (the level counts, then the group and work counts).
struct DevAlloc {
  virtual int alloc(void** p, size_t bytes) = 0;
  virtual ~DevAlloc() = default;
};
// Device buffers handed out in request order and kept for the next round of
// requests in the same order: a repeated build (time integration) finds its
// buffers in place and only a request that outgrows its slot reallocates it.
struct SeqPool {
  std::vector<void*> ptr;
  std::vector<size_t> cap;
  size_t next = 0;
  void* take(size_t bytes);  // nullptr when the device allocation fails
  void rewind() { next = 0; }
  SeqPool() = default;
  SeqPool(const SeqPool&) = delete;
  SeqPool& operator=(const SeqPool&) = delete;
  ~SeqPool();
};
// Scratch of the device build kept between builds: whole-build arrays,
// per-level arrays (the same slots every level) and the cell arrays.
struct BuildPools {
  SeqPool outer, level, cells;
  int last_levels = 0;  // non-empty levels of the previous build (0: unknown)
  void* pinned = nullptr;  // page-locked host copy of the build's scalars (tree_gpu.hip)
  BuildPools() = default;
  BuildPools(const BuildPools&) = delete;
  BuildPools& operator=(const BuildPools&) = delete;
  ~BuildPools();
};
struct DeviceArrays {
  const double* box = nullptr;     // [nc * 6]
  const double* mp64 = nullptr;    // [nc * 10]
  const float* geo_host = nullptr; // [nc * 4]
  const int32_t* depth = nullptr;  // [nc]
  const int32_t* groups = nullptr; // [ng]
};
// Inputs are host arrays (copied) or, with inputs_on_device, device arrays
// (checked on the device).
int build_device_tree(const float* pos_in, const float* mass_in, bool inputs_on_device, int64_t n,
                      int n_leaf, int n_group, HostTree& h, DevTree& dt, DeviceArrays& out,
                      DevAlloc& alloc, void* stream, std::string& err,
                      BuildPools* pools = nullptr);

// Leapfrog pieces: v += h a, x += dt v, and FP64 (1/2 sum m v^2, sum m v).
int launch_kick(float* vel, const float* acc, int64_t n, float h, void* stream);
int launch_drift(float* pos, const float* vel, int64_t n, float dt, void* stream);
int launch_kinetic(const float* mass, const float* vel, int64_t n, double* part, double* out4,
                   void* stream);
int64_t kinetic_scratch_entries();

int launch_diag(const DevTree& T, const float* acc, const float* pot, double* part_sums,
                double* out4, void* stream);
int64_t scan_scratch_entries(int64_t ng);
int64_t diag_scratch_entries(int64_t n);

// The file-scope device scratch array of octgrav_forces_noalloc: its size,
// and its device address on the current device (looked up on the first call
// per device, then cached).  0 on success.
size_t noalloc_scratch_bytes();
int noalloc_scratch(void** ptr, std::string& err);

}  // namespace octgrav
