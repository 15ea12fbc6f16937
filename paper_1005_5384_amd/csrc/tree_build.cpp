// Host octree construction (Sec. 2.1): root cube, octant subdivision down to
// leaves of at most n_leaf particles, tight boxes, boundary cubes, FP64
// monopole and traceless quadrupole moments, groups, and the FP32 device
// images.  Particles are ordered along 63-bit Morton keys (Z-order of the
// depth-21 octants, ties by input index), which also puts neighbouring groups
// next to each other in memory (the re-ordering described at the end of
// Sec. 2.1).  Cells are numbered breadth-first, so children are contiguous
// and a breadth-first walk meets cells in ascending id order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include <omp.h>

#include "octgrav_internal.h"

namespace octgrav {
namespace {

constexpr uint32_t kGridMax = (1u << kMaxDepth) - 1;

// Grid coordinate of x on one axis: the u in [0, 2^21) with
// corner + u*step <= x < corner + (u+1)*step, step = side / 2^21.  The
// floor gives it up to rounding of (x - corner); the two loops make it exact
// against the grid planes, which are the octants' splitting planes at every
// level (a particle on a plane belongs to the upper side).
inline uint32_t grid_coord(double x, double corner, double step, double inv_step) {
  double f = std::floor((x - corner) * inv_step);
  int64_t u = f < 0 ? 0 : (f > (double)kGridMax ? (int64_t)kGridMax : (int64_t)f);
  while (u > 0 && corner + (double)u * step > x) --u;
  while (u < (int64_t)kGridMax && corner + (double)(u + 1) * step <= x) ++u;
  return (uint32_t)u;
}

// Spreads the 21 bits of v to every third bit position.
inline uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

// Stable LSD radix sort of (key, idx) by key, 8 bits per pass, skipping
// passes whose digit is the same for every key.
void radix_sort(std::vector<uint64_t>& key, std::vector<int32_t>& idx) {
  const int64_t n = (int64_t)key.size();
  std::vector<uint64_t> k2(n);
  std::vector<int32_t> i2(n);
  const int nt = std::max(1, std::min(omp_get_max_threads(), (int)(n / 65536) + 1));
  std::vector<int64_t> hist((size_t)nt * 256);
  for (int pass = 0; pass < 8; ++pass) {
    const int sh = 8 * pass;
    std::fill(hist.begin(), hist.end(), 0);
#pragma omp parallel num_threads(nt)
    {
      int t = omp_get_thread_num();
      int64_t a = n * t / nt, b = n * (t + 1) / nt;
      int64_t* h = &hist[(size_t)t * 256];
      for (int64_t i = a; i < b; ++i) ++h[(key[i] >> sh) & 255];
    }
    int64_t single = 0;
    for (int d = 0; d < 256 && !single; ++d) {
      int64_t s = 0;
      for (int t = 0; t < nt; ++t) s += hist[(size_t)t * 256 + d];
      if (s == n) single = 1;
    }
    if (single) continue;
    int64_t run = 0;
    for (int d = 0; d < 256; ++d)
      for (int t = 0; t < nt; ++t) {
        int64_t c = hist[(size_t)t * 256 + d];
        hist[(size_t)t * 256 + d] = run;
        run += c;
      }
#pragma omp parallel num_threads(nt)
    {
      int t = omp_get_thread_num();
      int64_t a = n * t / nt, b = n * (t + 1) / nt;
      int64_t* h = &hist[(size_t)t * 256];
      for (int64_t i = a; i < b; ++i) {
        int64_t p = h[(key[i] >> sh) & 255]++;
        k2[p] = key[i];
        i2[p] = idx[i];
      }
    }
    key.swap(k2);
    idx.swap(i2);
  }
}

}  // namespace

bool validate_inputs(const float* pos, const float* mass, int64_t n, int n_leaf, int n_group,
                     std::string& err) {
  if (!pos || !mass) return err = "pos and mass must be non-NULL", false;
  if (n < 1 || n >= (int64_t(1) << 31)) return err = "n must satisfy 1 <= n < 2^31", false;
  if (n_leaf < 1 || n_leaf > 64) return err = "n_leaf must be in 1..64", false;
  if (n_group < 1 || n_group > 1024) return err = "n_group must be in 1..1024", false;
  const double lim = std::ldexp(1.0, 60);
  bool bad_pos = false, bad_mass = false;
#pragma omp parallel for reduction(|| : bad_pos, bad_mass)
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) {
      double v = pos[3 * i + k];
      bad_pos = bad_pos || !std::isfinite(v) || std::fabs(v) >= lim;
    }
    bad_mass = bad_mass || !std::isfinite(mass[i]) || !(mass[i] > 0.0f);
  }
  if (bad_pos) return err = "positions must be finite with |x| < 2^60", false;
  if (bad_mass) return err = "masses must be finite and > 0", false;
  return true;
}

void bounding_box(const float* pos, int64_t n, double lo[3], double hi[3]) {
  for (int k = 0; k < 3; ++k) {
    double a = pos[k], b = pos[k];
#pragma omp parallel for reduction(min : a) reduction(max : b)
    for (int64_t i = 0; i < n; ++i) {
      a = std::min(a, (double)pos[3 * i + k]);
      b = std::max(b, (double)pos[3 * i + k]);
    }
    lo[k] = a;
    hi[k] = b;
  }
}

// Root cube: centred on the bounding box, side the power of two S with
// ext < S <= 2 ext (S = 1 for a single point).
void root_cube(const double lo[3], const double hi[3], double corner[3], double* side) {
  double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
  int e = 1;
  if (ext > 0) std::frexp(ext, &e);
  *side = ext > 0 ? std::ldexp(1.0, e) : 1.0;
  for (int k = 0; k < 3; ++k) corner[k] = (lo[k] + hi[k]) * 0.5 - 0.5 * *side;
}

bool build_host_tree(const float* pos, const float* mass, int64_t n, int n_leaf, int n_group,
                     HostTree& T, std::string& err) {
  if (!validate_inputs(pos, mass, n, n_leaf, n_group, err)) return false;
  T = HostTree();
  T.n = n;
  T.n_leaf = n_leaf;
  T.n_group = n_group;

  double lo[3], hi[3];
  bounding_box(pos, n, lo, hi);
  root_cube(lo, hi, T.corner, &T.side);

  // Morton keys and the sort.
  const double step = std::ldexp(T.side, -kMaxDepth), inv = std::ldexp(1.0 / T.side, kMaxDepth);
  std::vector<uint64_t> key(n);
  std::vector<int32_t> idx(n);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    uint32_t u[3];
    for (int k = 0; k < 3; ++k) u[k] = grid_coord((double)pos[3 * i + k], T.corner[k], step, inv);
    key[i] = spread3(u[0]) | spread3(u[1]) << 1 | spread3(u[2]) << 2;
    idx[i] = (int32_t)i;
  }
  radix_sort(key, idx);
  T.perm = idx;

  // Level-synchronous subdivision in breadth-first order.
  std::vector<int64_t> cfirst{0}, cn{n};
  std::vector<int32_t> cdepth{0}, cparent{-1}, cfc{-1}, cnc{0};
  int64_t lbeg = 0, lend = 1;
  for (int L = 0; lbeg < lend; ++L) {
    const int64_t m = lend - lbeg;
    std::vector<int32_t> nkid(m, 0);
    std::vector<int64_t> kb((size_t)m * 9, 0);  // child digit boundaries
    const int sh = 3 * (kMaxDepth - 1 - L);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < m; ++j) {
      int64_t c = lbeg + j, a = cfirst[c], b = a + cn[c];
      if (cn[c] <= n_leaf || L == kMaxDepth) continue;
      int64_t* bd = &kb[(size_t)j * 9];
      bd[0] = a;
      for (int d = 1; d < 8; ++d)
        bd[d] = std::partition_point(key.begin() + bd[d - 1], key.begin() + b,
                                     [&](uint64_t kk) { return (int)((kk >> sh) & 7) < d; }) -
                key.begin();
      bd[8] = b;
      int cnt = 0;
      for (int d = 0; d < 8; ++d) cnt += bd[d + 1] > bd[d];
      nkid[j] = cnt;
    }
    int64_t next = lend;
    for (int64_t j = 0; j < m; ++j) {
      int64_t c = lbeg + j;
      if (!nkid[j]) continue;
      cfc[c] = (int32_t)next;
      cnc[c] = nkid[j];
      const int64_t* bd = &kb[(size_t)j * 9];
      for (int d = 0; d < 8; ++d)
        if (bd[d + 1] > bd[d]) {
          cfirst.push_back(bd[d]);
          cn.push_back(bd[d + 1] - bd[d]);
          cdepth.push_back(L + 1);
          cparent.push_back((int32_t)c);
          cfc.push_back(-1);
          cnc.push_back(0);
          ++next;
        }
    }
    T.max_level_cells = std::max(T.max_level_cells, m);
    if (next > lend) T.max_depth = L + 1;
    lbeg = lend;
    lend = next;
  }
  const int64_t nc = (int64_t)cfirst.size();

  // Sorted particle images.
  T.part.resize((size_t)n * 4);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    int32_t p = T.perm[i];
    for (int k = 0; k < 3; ++k) T.part[4 * i + k] = pos[3 * p + k];
    T.part[4 * i + 3] = mass[p];
  }

  // Boxes and moments, bottom-up by level (cells of one level are contiguous).
  T.topo.resize((size_t)nc * 4);
  T.depth.assign(cdepth.begin(), cdepth.end());
  T.box.resize((size_t)nc * 6);
  T.mp64.resize((size_t)nc * 10);
  std::vector<int64_t> lvl_start(T.max_depth + 2, nc);
  for (int64_t c = nc - 1; c >= 0; --c) lvl_start[cdepth[c]] = c;
  for (int L = T.max_depth; L >= 0; --L) {
    const int64_t a = lvl_start[L], b = lvl_start[L + 1];
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = a; c < b; ++c) {
      double* bx = &T.box[(size_t)c * 6];
      double* q = &T.mp64[(size_t)c * 10];
      if (cnc[c] == 0) {
        double M = 0, sx = 0, sy = 0, sz = 0;
        for (int k = 0; k < 3; ++k) {
          bx[k] = INFINITY;
          bx[3 + k] = -INFINITY;
        }
        for (int64_t i = cfirst[c]; i < cfirst[c] + cn[c]; ++i) {
          const float* p = &T.part[4 * i];
          for (int k = 0; k < 3; ++k) {
            bx[k] = std::min(bx[k], (double)p[k]);
            bx[3 + k] = std::max(bx[3 + k], (double)p[k]);
          }
          double w = p[3];
          M += w;
          sx += w * p[0];
          sy += w * p[1];
          sz += w * p[2];
        }
        double com[3] = {sx / M, sy / M, sz / M}, Q[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t i = cfirst[c]; i < cfirst[c] + cn[c]; ++i) {
          const float* p = &T.part[4 * i];
          double d0 = p[0] - com[0], d1 = p[1] - com[1], d2 = p[2] - com[2], w = p[3];
          double r2 = d0 * d0 + d1 * d1 + d2 * d2;
          Q[0] += w * (3 * d0 * d0 - r2);
          Q[1] += w * (3 * d1 * d1 - r2);
          Q[2] += w * (3 * d2 * d2 - r2);
          Q[3] += w * 3 * d0 * d1;
          Q[4] += w * 3 * d0 * d2;
          Q[5] += w * 3 * d1 * d2;
        }
        q[0] = M;
        for (int k = 0; k < 3; ++k) q[1 + k] = com[k];
        for (int k = 0; k < 6; ++k) q[4 + k] = Q[k];
      } else {
        double M = 0, sx = 0, sy = 0, sz = 0;
        for (int k = 0; k < 3; ++k) {
          bx[k] = INFINITY;
          bx[3 + k] = -INFINITY;
        }
        for (int64_t ch = cfc[c]; ch < cfc[c] + cnc[c]; ++ch) {
          const double* cb = &T.box[(size_t)ch * 6];
          const double* cq = &T.mp64[(size_t)ch * 10];
          for (int k = 0; k < 3; ++k) {
            bx[k] = std::min(bx[k], cb[k]);
            bx[3 + k] = std::max(bx[3 + k], cb[3 + k]);
          }
          M += cq[0];
          sx += cq[0] * cq[1];
          sy += cq[0] * cq[2];
          sz += cq[0] * cq[3];
        }
        double com[3] = {sx / M, sy / M, sz / M}, Q[6] = {0, 0, 0, 0, 0, 0};
        // Parallel-axis shift of each child's traceless quadrupole to the
        // parent's centre of mass.
        for (int64_t ch = cfc[c]; ch < cfc[c] + cnc[c]; ++ch) {
          const double* cq = &T.mp64[(size_t)ch * 10];
          double d0 = cq[1] - com[0], d1 = cq[2] - com[1], d2 = cq[3] - com[2], w = cq[0];
          double r2 = d0 * d0 + d1 * d1 + d2 * d2;
          Q[0] += cq[4] + w * (3 * d0 * d0 - r2);
          Q[1] += cq[5] + w * (3 * d1 * d1 - r2);
          Q[2] += cq[6] + w * (3 * d2 * d2 - r2);
          Q[3] += cq[7] + w * 3 * d0 * d1;
          Q[4] += cq[8] + w * 3 * d0 * d2;
          Q[5] += cq[9] + w * 3 * d1 * d2;
        }
        q[0] = M;
        for (int k = 0; k < 3; ++k) q[1 + k] = com[k];
        for (int k = 0; k < 6; ++k) q[4 + k] = Q[k];
      }
    }
  }

  // FP32 images: topology, boundary (centre of the tight box, side = its
  // largest extent), moments.
  T.geo.resize((size_t)nc * 4);
  T.mp.resize((size_t)nc * 12);
#pragma omp parallel for
  for (int64_t c = 0; c < nc; ++c) {
    int32_t* tp = &T.topo[(size_t)c * 4];
    tp[0] = cfc[c];
    tp[1] = cnc[c];
    tp[2] = (int32_t)cfirst[c];
    tp[3] = (int32_t)cn[c];
    const double* bx = &T.box[(size_t)c * 6];
    double l = 0;
    for (int k = 0; k < 3; ++k) {
      T.geo[4 * c + k] = (float)((bx[k] + bx[3 + k]) * 0.5);
      l = std::max(l, bx[3 + k] - bx[k]);
    }
    T.geo[4 * c + 3] = (float)l;
    const double* q = &T.mp64[(size_t)c * 10];
    float* f = &T.mp[(size_t)c * 12];
    f[0] = (float)q[1];
    f[1] = (float)q[2];
    f[2] = (float)q[3];
    f[3] = (float)q[0];
    f[4] = (float)q[4];
    f[5] = (float)q[5];
    f[6] = (float)q[6];
    f[7] = (float)q[7];
    f[8] = (float)q[8];
    f[9] = (float)q[9];
    f[10] = 0.0f;
    f[11] = 0.0f;
  }

  // Groups: the maximal cells with at most n_group particles, or leaves
  // (coincident particles at depth 21), ordered by first particle.
  for (int64_t c = 0; c < nc; ++c) {
    bool cand = cn[c] <= n_group || cnc[c] == 0;
    bool top = c == 0 || cn[cparent[c]] > n_group;
    if (cand && top) T.groups.push_back((int32_t)c);
  }
  std::sort(T.groups.begin(), T.groups.end(),
            [&](int32_t a, int32_t b) { return cfirst[a] < cfirst[b]; });
  const int64_t ng = (int64_t)T.groups.size();
  T.ginfo.resize((size_t)ng * 4);
  T.gbox.resize((size_t)ng * 8);
  for (int64_t g = 0; g < ng; ++g) {
    int32_t c = T.groups[g];
    T.ginfo[4 * g] = (int32_t)cfirst[c];
    T.ginfo[4 * g + 1] = (int32_t)cn[c];
    T.ginfo[4 * g + 2] = c;
    T.ginfo[4 * g + 3] = 0;
    const double* bx = &T.box[(size_t)c * 6];
    for (int k = 0; k < 3; ++k) {
      T.gbox[8 * g + k] = (float)bx[k];
      T.gbox[8 * g + 4 + k] = (float)bx[3 + k];
    }
    T.gbox[8 * g + 3] = 0.0f;
    T.gbox[8 * g + 7] = 0.0f;
    for (int32_t off = 0; off < cn[c]; off += kChunk) {
      T.work.push_back((int32_t)g);
      T.work.push_back(off);
    }
  }
  return true;
}

}  // namespace octgrav
