// TEST INFRASTRUCTURE ONLY.
//
// Plain, slow FP64 CPU oracle of the group tree-walk gravity method of
// Gaburov, Bedorf and Portegies Zwart, "Gravitational tree-code on graphics
// processing units: implementation in CUDA" (ICCS 2010).  Only the test suite,
// the smoke check and the CPU-baseline leg of the benchmark may load this
// library.  It shares no source, header, table or helper with the HIP library
// under test; the two meet only through seeded inputs.
//
// Readings of points the paper leaves open (fixed identically by the library
// under test, independently re-implemented there):
//   * Root cube (Sec. 2.1 "a cube containing all particles"): centred on the
//     bounding box, side S = 2^e with ext < S <= 2 ext (S = 1 if ext = 0).
//   * Subdivision (Sec. 2.1, Fig. "octree" caption): a cell is a leaf iff it
//     holds n <= n_leaf particles or sits at depth 21; otherwise its children
//     are its non-empty octants in octant order (x bit | y bit<<1 | z bit<<2);
//     a particle on a splitting plane goes to the upper octant.
//   * Particle order: Z-order of the depth-21 octants, ties by input index.
//   * Cells are numbered in breadth-first (level) order, root = 0.
//   * Boundary (Sec. 2.1 and Fig. "octree" caption): a cube centred on the
//     tight bounding box with side = the box's largest side.
//   * Groups (Sec. 2.1): the maximal cells holding n <= n_group particles, or
//     leaves (coincident particles at depth 21), ordered by first particle.
//   * Opening test (Sec. 2.2, the test-cell listing): the classic size over
//     distance criterion, with d measured from the boundary centre to the
//     nearest point of the group's bounding box, in FP32 without contraction.
//   * Which list gets what (Sec. 2.2, the test-cell listing): an opened leaf
//     goes to the leaf list, an unopened cell (leaf or node) to the cell list.
//   * Interactions (Sec. 2.3): Plummer-softened particle-particle forces and
//     potentials (self excluded), softened monopole plus traceless quadrupole
//     particle-cell forces and potentials about the centre of mass; G = 1.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include <omp.h>

#include "oracle_tree.h"

namespace orc {

// Octant of point p in the cube (corner, side): each coordinate goes to the
// upper half iff it is >= the cube's midplane.
int octant_of(const Tree& t, int32_t p, const double corner[3], double side) {
  int o = 0;
  for (int k = 0; k < 3; ++k) {
    double mid = corner[k] + 0.5 * side;
    if (t.x[k][p] >= mid) o |= (1 << k);
  }
  return o;
}

void child_corner(const double corner[3], double side, int oct, double out[3]) {
  for (int k = 0; k < 3; ++k) out[k] = corner[k] + (((oct >> k) & 1) ? 0.5 * side : 0.0);
}

// Puts the index range [a, b) into Z-order by recursive stable octant
// partitioning down to depth 21 (ties keep input order).
void zorder(Tree& t, int64_t a, int64_t b, const double corner[3], double side, int depth) {
  if (b - a <= 1 || depth == kMaxDepth) return;
  auto first = t.order.begin() + a, last = t.order.begin() + b;
  std::vector<int32_t> buckets[8];
  for (auto it = first; it != last; ++it) buckets[octant_of(t, *it, corner, side)].push_back(*it);
  int64_t pos = a;
  for (int o = 0; o < 8; ++o) {
    int64_t s = pos;
    for (int32_t p : buckets[o]) t.order[pos++] = p;
    double cc[3];
    child_corner(corner, side, o, cc);
    std::vector<int32_t>().swap(buckets[o]);
    zorder(t, s, pos, cc, 0.5 * side, depth + 1);
  }
}

// Temporary pointer tree built recursively, then renumbered breadth-first.
struct TNode {
  int64_t a, b;
  int depth;
  double corner[3], side;
  int kids[8];
  int nk = 0;
};

int make_node(Tree& t, std::vector<TNode>& pool, int64_t a, int64_t b, const double corner[3],
              double side, int depth) {
  int id = (int)pool.size();
  pool.push_back(TNode{});
  pool[id].a = a;
  pool[id].b = b;
  pool[id].depth = depth;
  pool[id].side = side;
  for (int k = 0; k < 3; ++k) pool[id].corner[k] = corner[k];
  if (b - a <= t.n_leaf || depth == kMaxDepth) return id;  // leaf
  // The range is in Z-order, so each non-empty octant is a contiguous run.
  int64_t s = a;
  while (s < b) {
    int o = octant_of(t, t.order[s], corner, side);
    int64_t e = s;
    while (e < b && octant_of(t, t.order[e], corner, side) == o) ++e;
    double cc[3];
    child_corner(corner, side, o, cc);
    int kid = make_node(t, pool, s, e, cc, 0.5 * side, depth + 1);
    pool[id].kids[pool[id].nk++] = kid;
    s = e;
  }
  return id;
}

void cell_properties(Tree& t, Cell& c) {
  for (int k = 0; k < 3; ++k) {
    c.mn[k] = INFINITY;
    c.mx[k] = -INFINITY;
  }
  double M = 0, mx = 0, my = 0, mz = 0;
  for (int64_t i = c.first; i < c.first + c.n; ++i) {
    int32_t p = t.order[i];
    for (int k = 0; k < 3; ++k) {
      c.mn[k] = std::min(c.mn[k], t.x[k][p]);
      c.mx[k] = std::max(c.mx[k], t.x[k][p]);
    }
    M += t.m[p];
    mx += t.m[p] * t.x[0][p];
    my += t.m[p] * t.x[1][p];
    mz += t.m[p] * t.x[2][p];
  }
  c.l = 0;
  for (int k = 0; k < 3; ++k) {
    c.cb[k] = (c.mn[k] + c.mx[k]) * 0.5;
    c.l = std::max(c.l, c.mx[k] - c.mn[k]);
  }
  c.M = M;
  c.com[0] = mx / M;
  c.com[1] = my / M;
  c.com[2] = mz / M;
  // Traceless quadrupole about the centre of mass: sum m (3 s_j s_k - |s|^2 delta_jk).
  for (double& q : c.Q) q = 0;
  for (int64_t i = c.first; i < c.first + c.n; ++i) {
    int32_t p = t.order[i];
    double s0 = t.x[0][p] - c.com[0], s1 = t.x[1][p] - c.com[1], s2 = t.x[2][p] - c.com[2];
    double ss = s0 * s0 + s1 * s1 + s2 * s2, w = t.m[p];
    c.Q[0] += w * (3 * s0 * s0 - ss);
    c.Q[1] += w * (3 * s1 * s1 - ss);
    c.Q[2] += w * (3 * s2 * s2 - ss);
    c.Q[3] += w * 3 * s0 * s1;
    c.Q[4] += w * 3 * s0 * s2;
    c.Q[5] += w * 3 * s1 * s2;
  }
  for (int k = 0; k < 3; ++k) c.geo[k] = (float)c.cb[k];
  c.geo[3] = (float)c.l;
}

void find_groups(const Tree& t, int c, std::vector<int32_t>& out) {
  const Cell& cell = t.cells[c];
  if (cell.n <= t.n_group || cell.n_child == 0) {
    out.push_back(c);
    return;
  }
  for (int k = 0; k < cell.n_child; ++k) find_groups(t, cell.first_child + k, out);
}

Tree* build(const float* pos, const float* mass, int64_t n, int n_leaf, int n_group) {
  Tree* t = new Tree;
  t->n = n;
  t->n_leaf = n_leaf;
  t->n_group = n_group;
  for (int k = 0; k < 3; ++k) t->x[k].resize(n);
  t->m.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) t->x[k][i] = (double)pos[3 * i + k];
    t->m[i] = (double)mass[i];
  }
  // Root cube: centred on the bounding box, power-of-two side exceeding its extent.
  double lo[3], hi[3], ext = 0;
  for (int k = 0; k < 3; ++k) {
    lo[k] = *std::min_element(t->x[k].begin(), t->x[k].end());
    hi[k] = *std::max_element(t->x[k].begin(), t->x[k].end());
    ext = std::max(ext, hi[k] - lo[k]);
  }
  if (ext == 0) {
    t->S = 1.0;
  } else {
    int e;
    std::frexp(ext, &e);
    t->S = std::ldexp(1.0, e);
  }
  for (int k = 0; k < 3; ++k) t->L[k] = (lo[k] + hi[k]) * 0.5 - 0.5 * t->S;

  t->order.resize(n);
  for (int64_t i = 0; i < n; ++i) t->order[i] = (int32_t)i;
  zorder(*t, 0, n, t->L, t->S, 0);

  std::vector<TNode> pool;
  pool.reserve(2 * (size_t)(n / std::max(1, n_leaf)) + 64);
  make_node(*t, pool, 0, n, t->L, t->S, 0);

  // Breadth-first renumbering; the children of each cell become contiguous.
  std::vector<int> queue{0}, parent{-1};
  for (size_t h = 0; h < queue.size(); ++h)
    for (int k = 0; k < pool[queue[h]].nk; ++k) {
      queue.push_back(pool[queue[h]].kids[k]);
      parent.push_back((int)h);
    }
  t->cells.resize(queue.size());
  std::vector<int> bfs_id(pool.size());
  for (size_t h = 0; h < queue.size(); ++h) bfs_id[queue[h]] = (int)h;
  for (size_t h = 0; h < queue.size(); ++h) {
    const TNode& tn = pool[queue[h]];
    Cell& c = t->cells[h];
    c.first = tn.a;
    c.n = tn.b - tn.a;
    c.depth = tn.depth;
    c.parent = parent[h];
    c.side = tn.side;
    for (int k = 0; k < 3; ++k) c.corner[k] = tn.corner[k];
    c.n_child = tn.nk;
    c.first_child = tn.nk ? bfs_id[tn.kids[0]] : -1;
    t->max_depth = std::max(t->max_depth, tn.depth);
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t h = 0; h < (int64_t)t->cells.size(); ++h) cell_properties(*t, t->cells[h]);

  find_groups(*t, 0, t->groups);
  std::sort(t->groups.begin(), t->groups.end(),
            [&](int32_t a, int32_t b) { return t->cells[a].first < t->cells[b].first; });
  return t;
}

// Opening test in FP32 with this exact operation sequence (no contraction):
// t_k = max(max(gmin_k - cb_k, cb_k - gmax_k), 0); d2 = (tx^2 + ty^2) + tz^2;
// open iff d2 == 0 or d2 * theta^2 < l^2.
bool mac_open(const float gmin[3], const float gmax[3], const float geo[4], float th2) {
  float tt[3];
  for (int k = 0; k < 3; ++k) {
    float a = gmin[k] - geo[k];
    float b = geo[k] - gmax[k];
    float m = a > b ? a : b;
    tt[k] = m > 0.0f ? m : 0.0f;
  }
  float sx = tt[0] * tt[0];
  float sy = tt[1] * tt[1];
  float sz = tt[2] * tt[2];
  float d2 = (sx + sy) + sz;
  float lhs = d2 * th2;
  float rhs = geo[3] * geo[3];
  return d2 == 0.0f || lhs < rhs;
}

void group_box(const Tree& t, int32_t gcell, float gmin[3], float gmax[3]) {
  const Cell& g = t.cells[gcell];
  // Exact: the tight box of FP32 positions is made of FP32 values.
  for (int k = 0; k < 3; ++k) {
    gmin[k] = (float)g.mn[k];
    gmax[k] = (float)g.mx[k];
  }
}

// Stack walk of one group (the tree-walk and test-cell listings of Sec. 2.2),
// returning its cell list and leaf list in canonical ascending order.
void walk_group(const Tree& t, int32_t gcell, float theta, std::vector<int32_t>& C,
                std::vector<int32_t>& Lv) {
  C.clear();
  Lv.clear();
  if (t.cells[0].n_child == 0) {
    Lv.push_back(0);
    return;
  }
  float th2 = theta * theta;
  float gmin[3], gmax[3];
  group_box(t, gcell, gmin, gmax);
  std::vector<int32_t> stack{0};
  while (!stack.empty()) {
    int32_t node = stack.back();
    stack.pop_back();
    const Cell& nc = t.cells[node];
    for (int k = 0; k < nc.n_child; ++k) {
      int32_t c = nc.first_child + k;
      if (mac_open(gmin, gmax, t.cells[c].geo, th2)) {
        if (t.cells[c].n_child == 0)
          Lv.push_back(c);
        else
          stack.push_back(c);
      } else {
        C.push_back(c);
      }
    }
  }
  std::sort(C.begin(), C.end());
  std::sort(Lv.begin(), Lv.end());
}

// The same lists from their definition, without a walk: c is in the cell
// list iff every proper ancestor of c is opened and c is not; a leaf is in
// the leaf list iff it and every proper ancestor are opened.  The root is
// always opened.
void brute_group(const Tree& t, int32_t gcell, float theta, std::vector<int32_t>& C,
                 std::vector<int32_t>& Lv) {
  C.clear();
  Lv.clear();
  float th2 = theta * theta;
  float gmin[3], gmax[3];
  group_box(t, gcell, gmin, gmax);
  int nc = (int)t.cells.size();
  std::vector<char> opened(nc);
  for (int c = 0; c < nc; ++c) opened[c] = (c == 0) ? 1 : mac_open(gmin, gmax, t.cells[c].geo, th2);
  for (int c = 0; c < nc; ++c) {
    bool anc = true;
    for (int a = t.cells[c].parent; a >= 0; a = t.cells[a].parent) anc = anc && opened[a];
    if (!anc) continue;
    if (!opened[c]) C.push_back(c);
    else if (t.cells[c].n_child == 0) Lv.push_back(c);
  }
}

typedef void (*walk_fn)(const Tree&, int32_t, float, std::vector<int32_t>&, std::vector<int32_t>&);

// CSR lists of the selected groups (sel: group indices, NULL = every group
// in order), in the order given.
int lists_impl(const Tree& t, float theta, walk_fn fn, int64_t* c_off, int32_t* c_ids,
               int64_t* l_off, int32_t* l_ids, int64_t* n_c, int64_t* n_l,
               const int32_t* sel = nullptr, int64_t n_sel = -1) {
  const int64_t ngt = (int64_t)t.groups.size();
  if (sel)
    for (int64_t u = 0; u < n_sel; ++u)
      if (sel[u] < 0 || sel[u] >= ngt) return -1;
  const int64_t ng = sel ? n_sel : ngt;
  std::vector<std::vector<int32_t>> C(ng), Lv(ng);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < ng; ++g) fn(t, t.groups[sel ? sel[g] : g], theta, C[g], Lv[g]);
  int64_t sc = 0, sl = 0;
  for (int64_t g = 0; g < ng; ++g) {
    if (c_off) c_off[g] = sc;
    if (l_off) l_off[g] = sl;
    if (c_ids) std::copy(C[g].begin(), C[g].end(), c_ids + sc);
    if (l_ids) std::copy(Lv[g].begin(), Lv[g].end(), l_ids + sl);
    sc += (int64_t)C[g].size();
    sl += (int64_t)Lv[g].size();
  }
  if (c_off) c_off[ng] = sc;
  if (l_off) l_off[ng] = sl;
  if (n_c) *n_c = sc;
  if (n_l) *n_l = sl;
  return 0;
}

// Offset variant of the opening test (Barnes' criterion with the boundary
// side as the size; the paper's choice of centre leaves this open): d from the
// cell's FP32 centre of mass com to the group box, the size enlarged by
// theta times the offset delta = |com - cb|, all in FP32 without contraction
// and a correctly rounded square root:
//   delta = sqrt((dx*dx + dy*dy) + dz*dz), d = com - cb;  l' = l + theta*delta;
//   open iff d2 == 0 or d2 * theta^2 < l'^2   (d2 as in mac_open, about com).
bool mac_open_com(const float gmin[3], const float gmax[3], const float com[3], const float geo[4],
                  float theta) {
  float dx = com[0] - geo[0], dy = com[1] - geo[1], dz = com[2] - geo[2];
  float px = dx * dx, py = dy * dy, pz = dz * dz;
  float delta = std::sqrt((px + py) + pz);
  float td = theta * delta;
  float g[4] = {com[0], com[1], com[2], geo[3] + td};
  return mac_open(gmin, gmax, g, theta * theta);
}

// The tree walk (as walk_group) and the walk-free characterisation (as
// brute_group) under the offset test; com is [n_cells x 3] FP32.
void walk_group_com(const Tree& t, int32_t gcell, float theta, const float* com,
                    std::vector<int32_t>& C, std::vector<int32_t>& Lv) {
  C.clear();
  Lv.clear();
  if (t.cells[0].n_child == 0) {
    Lv.push_back(0);
    return;
  }
  float gmin[3], gmax[3];
  group_box(t, gcell, gmin, gmax);
  std::vector<int32_t> stack{0};
  while (!stack.empty()) {
    const Cell& nc = t.cells[stack.back()];
    stack.pop_back();
    for (int k = 0; k < nc.n_child; ++k) {
      int32_t c = nc.first_child + k;
      if (mac_open_com(gmin, gmax, com + 3 * (int64_t)c, t.cells[c].geo, theta)) {
        if (t.cells[c].n_child == 0)
          Lv.push_back(c);
        else
          stack.push_back(c);
      } else {
        C.push_back(c);
      }
    }
  }
  std::sort(C.begin(), C.end());
  std::sort(Lv.begin(), Lv.end());
}

void brute_group_com(const Tree& t, int32_t gcell, float theta, const float* com,
                     std::vector<int32_t>& C, std::vector<int32_t>& Lv) {
  C.clear();
  Lv.clear();
  float gmin[3], gmax[3];
  group_box(t, gcell, gmin, gmax);
  int nc = (int)t.cells.size();
  std::vector<char> opened(nc);
  for (int c = 0; c < nc; ++c)
    opened[c] = (c == 0) ? 1 : mac_open_com(gmin, gmax, com + 3 * (int64_t)c, t.cells[c].geo, theta);
  for (int c = 0; c < nc; ++c) {
    bool anc = true;
    for (int a = t.cells[c].parent; a >= 0; a = t.cells[a].parent) anc = anc && opened[a];
    if (!anc) continue;
    if (!opened[c]) C.push_back(c);
    else if (t.cells[c].n_child == 0) Lv.push_back(c);
  }
}

// FP64 evaluation of one group's lists for each of its particles (Sec. 2.3).
void eval_group(const Tree& t, int32_t gcell, const std::vector<int32_t>& C,
                const std::vector<int32_t>& Lv, double eps2, double* acc, double* pot) {
  const Cell& g = t.cells[gcell];
  for (int64_t ii = g.first; ii < g.first + g.n; ++ii) {
    int32_t i = t.order[ii];
    double xi = t.x[0][i], yi = t.x[1][i], zi = t.x[2][i];
    double ax = 0, ay = 0, az = 0, ph = 0;
    for (int32_t c : C) {  // particle-cell: monopole + traceless quadrupole
      const Cell& cc = t.cells[c];
      double R0 = xi - cc.com[0], R1 = yi - cc.com[1], R2 = zi - cc.com[2];
      double r2 = R0 * R0 + R1 * R1 + R2 * R2 + eps2;
      double ri = 1.0 / std::sqrt(r2);
      double ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
      const double* Q = cc.Q;
      double q0 = Q[0] * R0 + Q[3] * R1 + Q[4] * R2;
      double q1 = Q[3] * R0 + Q[1] * R1 + Q[5] * R2;
      double q2 = Q[4] * R0 + Q[5] * R1 + Q[2] * R2;
      double s = R0 * q0 + R1 * q1 + R2 * q2;
      ph += -cc.M * ri - 0.5 * s * ri5;
      ax += -cc.M * R0 * ri3 + q0 * ri5 - 2.5 * s * R0 * ri7;
      ay += -cc.M * R1 * ri3 + q1 * ri5 - 2.5 * s * R1 * ri7;
      az += -cc.M * R2 * ri3 + q2 * ri5 - 2.5 * s * R2 * ri7;
    }
    for (int32_t lf : Lv) {  // particle-particle over the leaf's particles
      const Cell& lc = t.cells[lf];
      for (int64_t jj = lc.first; jj < lc.first + lc.n; ++jj) {
        int32_t j = t.order[jj];
        if (j == i) continue;
        double R0 = t.x[0][j] - xi, R1 = t.x[1][j] - yi, R2 = t.x[2][j] - zi;
        double r2 = R0 * R0 + R1 * R1 + R2 * R2 + eps2;
        double ri = 1.0 / std::sqrt(r2);
        double mri3 = t.m[j] * ri * ri * ri;
        ax += mri3 * R0;
        ay += mri3 * R1;
        az += mri3 * R2;
        ph -= t.m[j] * ri;
      }
    }
    acc[3 * i + 0] = ax;
    acc[3 * i + 1] = ay;
    acc[3 * i + 2] = az;
    if (pot) pot[i] = ph;
  }
}

}  // namespace orc

using namespace orc;

extern "C" {

// Plain FP64 direct summation (the exact force the paper's accuracy metric
// compares against, Sec. 3.1): a_i = sum_{j!=i} m_j (x_j-x_i)/(r^2+eps^2)^{3/2},
// phi_i = -sum_{j!=i} m_j/(r^2+eps^2)^{1/2}.  targets == NULL means all;
// results are written in target order (acc nt x 3, pot nt).
int orc_direct(const float* pos, const float* mass, int64_t n, float eps, const int64_t* targets,
               int64_t nt, double* acc, double* pot) {
  if (!pos || !mass || n < 1 || !acc) return -1;
  if (!targets) nt = n;
  double eps2 = (double)eps * (double)eps;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t u = 0; u < nt; ++u) {
    int64_t i = targets ? targets[u] : u;
    double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    double ax = 0, ay = 0, az = 0, ph = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double R0 = (double)pos[3 * j] - xi, R1 = (double)pos[3 * j + 1] - yi,
             R2 = (double)pos[3 * j + 2] - zi;
      double r2 = R0 * R0 + R1 * R1 + R2 * R2 + eps2;
      double ri = 1.0 / std::sqrt(r2);
      double mri3 = (double)mass[j] * ri * ri * ri;
      ax += mri3 * R0;
      ay += mri3 * R1;
      az += mri3 * R2;
      ph -= (double)mass[j] * ri;
    }
    acc[3 * u] = ax;
    acc[3 * u + 1] = ay;
    acc[3 * u + 2] = az;
    if (pot) pot[u] = ph;
  }
  return 0;
}

void* orc_tree_build(const float* pos, const float* mass, int64_t n, int n_leaf, int n_group) {
  if (!pos || !mass || n < 1 || n_leaf < 1 || n_group < 1) return nullptr;
  return build(pos, mass, n, n_leaf, n_group);
}

void orc_tree_free(void* h) { delete (Tree*)h; }

// sizes: [n, n_cells, n_leaves, n_groups, max_depth]
int orc_tree_sizes(const void* h, int64_t* out) {
  const Tree& t = *(const Tree*)h;
  int64_t leaves = 0;
  for (const Cell& c : t.cells) leaves += (c.n_child == 0);
  out[0] = t.n;
  out[1] = (int64_t)t.cells.size();
  out[2] = leaves;
  out[3] = (int64_t)t.groups.size();
  out[4] = t.max_depth;
  return 0;
}

// Exports (any pointer may be NULL):
//   order  [n]        oracle position -> input index
//   topo   [nc x 4]   first_child, n_child, first particle, n particles
//   geo    [nc x 4]   FP32 boundary centre and side
//   mp     [nc x 10]  FP64 M, com xyz, Q xx yy zz xy xz yz
//   box    [nc x 6]   FP64 tight box min xyz, max xyz
//   depth  [nc]       level of each cell
//   groups [ng]       cell id of each group
//   cube   [4]        root cube corner xyz and side
int orc_tree_export(const void* h, int32_t* order, int32_t* topo, float* geo, double* mp,
                    double* box, int32_t* depth, int32_t* groups, double* cube) {
  const Tree& t = *(const Tree*)h;
  if (order) std::copy(t.order.begin(), t.order.end(), order);
  for (size_t c = 0; c < t.cells.size(); ++c) {
    const Cell& cc = t.cells[c];
    if (topo) {
      topo[4 * c] = cc.first_child;
      topo[4 * c + 1] = cc.n_child;
      topo[4 * c + 2] = (int32_t)cc.first;
      topo[4 * c + 3] = (int32_t)cc.n;
    }
    if (geo)
      for (int k = 0; k < 4; ++k) geo[4 * c + k] = cc.geo[k];
    if (mp) {
      mp[10 * c] = cc.M;
      for (int k = 0; k < 3; ++k) mp[10 * c + 1 + k] = cc.com[k];
      for (int k = 0; k < 6; ++k) mp[10 * c + 4 + k] = cc.Q[k];
    }
    if (box)
      for (int k = 0; k < 3; ++k) {
        box[6 * c + k] = cc.mn[k];
        box[6 * c + 3 + k] = cc.mx[k];
      }
    if (depth) depth[c] = cc.depth;
  }
  if (groups) std::copy(t.groups.begin(), t.groups.end(), groups);
  if (cube) {
    for (int k = 0; k < 3; ++k) cube[k] = t.L[k];
    cube[3] = t.S;
  }
  return 0;
}

// Per-cell octree cube: corner xyz and side [nc x 4] (FP64).
int orc_tree_cubes(const void* h, double* cubes) {
  const Tree& t = *(const Tree*)h;
  for (size_t c = 0; c < t.cells.size(); ++c) {
    for (int k = 0; k < 3; ++k) cubes[4 * c + k] = t.cells[c].corner[k];
    cubes[4 * c + 3] = t.cells[c].side;
  }
  return 0;
}

// Multipole (monopole + traceless quadrupole about the centre of mass) of an
// arbitrary particle set, evaluated at one target point with the same
// particle-cell formula the tree evaluation uses.  use_quad = 0 drops Q.
// out = {ax, ay, az, phi}.
int orc_multipole_eval(const float* pos, const float* mass, int64_t n, const double* target,
                       float eps, int use_quad, double* out) {
  Tree t;
  t.n = n;
  for (int k = 0; k < 3; ++k) t.x[k].resize(n);
  t.m.resize(n);
  t.order.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) t.x[k][i] = (double)pos[3 * i + k];
    t.m[i] = (double)mass[i];
    t.order[i] = (int32_t)i;
  }
  Cell c;
  c.first = 0;
  c.n = n;
  cell_properties(t, c);
  if (!use_quad)
    for (double& q : c.Q) q = 0;
  t.cells.push_back(c);
  // A one-particle "group" at the target sees this cell through the p-c path.
  t.x[0].push_back(target[0]);
  t.x[1].push_back(target[1]);
  t.x[2].push_back(target[2]);
  t.m.push_back(1.0);
  t.order.push_back((int32_t)n);
  Cell g;
  g.first = n;
  g.n = 1;
  t.cells.push_back(g);
  std::vector<int32_t> C{0}, Lv;
  std::vector<double> acc(3 * (n + 1)), pot(n + 1);
  eval_group(t, 1, C, Lv, (double)eps * (double)eps, acc.data(), pot.data());
  for (int k = 0; k < 3; ++k) out[k] = acc[3 * n + k];
  out[3] = pot[n];
  return 0;
}

int orc_mac_open(const float* gmin, const float* gmax, const float* geo, float theta) {
  float th2 = theta * theta;
  return mac_open(gmin, gmax, geo, th2) ? 1 : 0;
}

// Interaction lists of every group (CSR over groups, ascending ids).  NULL
// arrays give the sizes only.
int orc_lists(const void* h, float theta, int64_t* c_off, int32_t* c_ids, int64_t* l_off,
              int32_t* l_ids, int64_t* n_c, int64_t* n_l) {
  return lists_impl(*(const Tree*)h, theta, walk_group, c_off, c_ids, l_off, l_ids, n_c, n_l);
}

// The lists of the n_sel groups sel (group indices), CSR in that order
// (c_off, l_off have n_sel + 1 entries).  -1 if an index is out of range.
int orc_lists_groups(const void* h, float theta, const int32_t* sel, int64_t n_sel, int64_t* c_off,
                     int32_t* c_ids, int64_t* l_off, int32_t* l_ids, int64_t* n_c, int64_t* n_l) {
  if (!sel || n_sel < 0) return -1;
  return lists_impl(*(const Tree*)h, theta, walk_group, c_off, c_ids, l_off, l_ids, n_c, n_l, sel,
                    n_sel);
}

int orc_lists_brute(const void* h, float theta, int64_t* c_off, int32_t* c_ids, int64_t* l_off,
                    int32_t* l_ids, int64_t* n_c, int64_t* n_l) {
  return lists_impl(*(const Tree*)h, theta, brute_group, c_off, c_ids, l_off, l_ids, n_c, n_l);
}

// Single offset test (see mac_open_com): 1 = open.
int orc_mac_open_com(const float* gmin, const float* gmax, const float* com, const float* geo,
                     float theta) {
  return mac_open_com(gmin, gmax, com, geo, theta) ? 1 : 0;
}

// Lists under the offset test (brute != 0: from the walk-free
// characterisation); com is the FP32 centre of mass of every cell [nc x 3].
int orc_lists_com(const void* h, float theta, const float* com, int brute, int64_t* c_off,
                  int32_t* c_ids, int64_t* l_off, int32_t* l_ids, int64_t* n_c, int64_t* n_l) {
  const Tree& t = *(const Tree*)h;
  int64_t ng = (int64_t)t.groups.size();
  std::vector<std::vector<int32_t>> C(ng), Lv(ng);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < ng; ++g) {
    if (brute)
      brute_group_com(t, t.groups[g], theta, com, C[g], Lv[g]);
    else
      walk_group_com(t, t.groups[g], theta, com, C[g], Lv[g]);
  }
  int64_t sc = 0, sl = 0;
  for (int64_t g = 0; g < ng; ++g) {
    if (c_off) c_off[g] = sc;
    if (l_off) l_off[g] = sl;
    if (c_ids) std::copy(C[g].begin(), C[g].end(), c_ids + sc);
    if (l_ids) std::copy(Lv[g].begin(), Lv[g].end(), l_ids + sl);
    sc += (int64_t)C[g].size();
    sl += (int64_t)Lv[g].size();
  }
  if (c_off) c_off[ng] = sc;
  if (l_off) l_off[ng] = sl;
  if (n_c) *n_c = sc;
  if (n_l) *n_l = sl;
  return 0;
}

// Same-tree forces: walk + FP64 evaluation for the particles of the selected
// groups (sel == NULL: all groups).  acc [n x 3], pot [n] are indexed by input
// index; entries of unselected particles are left untouched.
int orc_forces(const void* h, float theta, float eps, const int32_t* sel, int64_t n_sel,
               double* acc, double* pot) {
  const Tree& t = *(const Tree*)h;
  if (!acc) return -1;
  int64_t ng = sel ? n_sel : (int64_t)t.groups.size();
  double eps2 = (double)eps * (double)eps;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t u = 0; u < ng; ++u) {
    int32_t gc = t.groups[sel ? sel[u] : u];
    std::vector<int32_t> C, Lv;
    walk_group(t, gc, theta, C, Lv);
    eval_group(t, gc, C, Lv, eps2, acc, pot);
  }
  return 0;
}

// FP64 forces of the selected groups (all: sel == NULL) from given CSR lists
// (cell ids; e.g. lists of another acceptance criterion), as orc_forces
// evaluates its own walk's lists.
int orc_forces_lists(const void* h, float eps, const int64_t* c_off, const int32_t* c_ids,
                     const int64_t* l_off, const int32_t* l_ids, const int32_t* sel, int64_t n_sel,
                     double* acc, double* pot) {
  const Tree& t = *(const Tree*)h;
  if (!acc) return -1;
  int64_t ng = sel ? n_sel : (int64_t)t.groups.size();
  double eps2 = (double)eps * (double)eps;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t u = 0; u < ng; ++u) {
    const int64_t g = sel ? sel[u] : u;
    std::vector<int32_t> C(c_ids + c_off[g], c_ids + c_off[g + 1]);
    std::vector<int32_t> Lv(l_ids + l_off[g], l_ids + l_off[g + 1]);
    eval_group(t, t.groups[g], C, Lv, eps2, acc, pot);
  }
  return 0;
}

// Kick-drift-kick leapfrog with FP64 direct-sum accelerations (the plain
// definitions: Plummer-softened Newtonian gravity, G = 1; v += a dt/2,
// x += v dt, v += a dt/2 with a from the new positions).  State in FP64;
// energy[2k], energy[2k + 1] = K, W after k steps (k = 0 .. steps).
namespace {
void acc64(const std::vector<double>& x, const double* m, int64_t n, double eps2,
           std::vector<double>& a, double* W) {
  double w = 0;
#pragma omp parallel for schedule(static) reduction(+ : w)
  for (int64_t i = 0; i < n; ++i) {
    double ax = 0, ay = 0, az = 0, ph = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = x[3 * j] - x[3 * i], dy = x[3 * j + 1] - x[3 * i + 1],
                   dz = x[3 * j + 2] - x[3 * i + 2];
      const double r2 = dx * dx + dy * dy + dz * dz + eps2, ri = 1.0 / std::sqrt(r2);
      const double f = m[j] * ri * ri * ri;
      ax += f * dx;
      ay += f * dy;
      az += f * dz;
      ph -= m[j] * ri;
    }
    a[3 * i] = ax;
    a[3 * i + 1] = ay;
    a[3 * i + 2] = az;
    w += 0.5 * m[i] * ph;
  }
  *W = w;
}
double kinetic(const std::vector<double>& v, const double* m, int64_t n) {
  double k = 0;
  for (int64_t i = 0; i < n; ++i)
    k += 0.5 * m[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
  return k;
}
}  // namespace

int orc_leapfrog(const double* pos, const double* vel, const double* mass, int64_t n, double eps,
                 double dt, int64_t steps, double* pos_out, double* vel_out, double* energy) {
  std::vector<double> x(pos, pos + 3 * n), v(vel, vel + 3 * n), a(3 * n);
  const double eps2 = eps * eps;
  double W;
  acc64(x, mass, n, eps2, a, &W);
  if (energy) {
    energy[0] = kinetic(v, mass, n);
    energy[1] = W;
  }
  for (int64_t s = 0; s < steps; ++s) {
    for (int64_t i = 0; i < 3 * n; ++i) v[i] += 0.5 * dt * a[i];
    for (int64_t i = 0; i < 3 * n; ++i) x[i] += dt * v[i];
    acc64(x, mass, n, eps2, a, &W);
    for (int64_t i = 0; i < 3 * n; ++i) v[i] += 0.5 * dt * a[i];
    if (energy) {
      energy[2 * (s + 1)] = kinetic(v, mass, n);
      energy[2 * (s + 1) + 1] = W;
    }
  }
  std::copy(x.begin(), x.end(), pos_out);
  std::copy(v.begin(), v.end(), vel_out);
  return 0;
}

// Interaction counts of the selected groups: per group |C_g|, |L_g| and the
// number of source particles in L_g.
int orc_counts(const void* h, float theta, int64_t* out3) {
  const Tree& t = *(const Tree*)h;
  int64_t ng = (int64_t)t.groups.size();
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < ng; ++g) {
    std::vector<int32_t> C, Lv;
    walk_group(t, t.groups[g], theta, C, Lv);
    int64_t np = 0;
    for (int32_t lf : Lv) np += t.cells[lf].n;
    out3[3 * g] = (int64_t)C.size();
    out3[3 * g + 1] = (int64_t)Lv.size();
    out3[3 * g + 2] = np;
  }
  return 0;
}

// FP64 diagnostics: total momentum sum m_i a_i and W = 1/2 sum m_i phi_i.
int orc_diagnostics(const float* mass, const double* acc, const double* pot, int64_t n,
                    double* out4) {
  double p0 = 0, p1 = 0, p2 = 0, w = 0;
  for (int64_t i = 0; i < n; ++i) {
    p0 += (double)mass[i] * acc[3 * i];
    p1 += (double)mass[i] * acc[3 * i + 1];
    p2 += (double)mass[i] * acc[3 * i + 2];
    if (pot) w += 0.5 * (double)mass[i] * pot[i];
  }
  out4[0] = p0;
  out4[1] = p1;
  out4[2] = p2;
  out4[3] = w;
  return 0;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

// Threads of the oracle's parallel loops from now on (k >= 1).
void orc_set_threads(int k) { omp_set_num_threads(k < 1 ? 1 : k); }

}  // extern "C"
