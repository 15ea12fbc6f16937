// TEST INFRASTRUCTURE ONLY: the oracle's own tree types, shared by the
// oracle's sources (oracle.cpp, oracle_mac.cpp) and nothing else.
#pragma once

#include <cstdint>
#include <vector>

namespace orc {

constexpr int kMaxDepth = 21;

struct Cell {
  int64_t first = 0, n = 0;  // contiguous range of the oracle's particle order
  int depth = 0, parent = -1;
  int first_child = -1, n_child = 0;
  double corner[3] = {0, 0, 0}, side = 0;  // the octree cube of this cell
  double mn[3], mx[3];                     // tight bounding box
  double cb[3], l;                         // boundary cube: centre and side
  double M, com[3], Q[6];                  // Q: xx, yy, zz, xy, xz, yz
  float geo[4];                            // FP32 boundary: the opening-test input
};

struct Tree {
  int64_t n = 0;
  int n_leaf = 0, n_group = 0;
  std::vector<double> x[3], m;
  std::vector<int32_t> order;  // oracle order position -> input index
  std::vector<Cell> cells;     // breadth-first order
  std::vector<int32_t> groups; // group cell ids, ascending first particle
  double L[3] = {0, 0, 0}, S = 1;
  int max_depth = 0;
};

bool mac_open(const float gmin[3], const float gmax[3], const float geo[4], float th2);
void group_box(const Tree& t, int32_t gcell, float gmin[3], float gmax[3]);
void walk_group(const Tree& t, int32_t gcell, float theta, std::vector<int32_t>& C,
                std::vector<int32_t>& Lv);
void eval_group(const Tree& t, int32_t gcell, const std::vector<int32_t>& C,
                const std::vector<int32_t>& Lv, double eps2, double* acc, double* pot);

}  // namespace orc
