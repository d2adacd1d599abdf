// Level-restricted adaptive octree (host). Section 4 (opening) of the paper: split a box
// into eight while it holds more than s points; then split coarser leaves until leaves
// that share a boundary point differ by at most one level.
#pragma once

#include <cstdint>
#include <unordered_map>
#include <vector>

namespace fmmlu {

constexpr int kDepth = 21;  // quantisation bits per axis

uint64_t morton3(uint32_t x, uint32_t y, uint32_t z);

struct Octree {
  int64_t n = 0;
  int leaf_size = 0;
  double root_lo[3] = {0, 0, 0};
  double side = 1.0;
  int nlevels = 0;

  // boxes
  std::vector<int8_t> level;
  std::vector<int32_t> cx, cy, cz;
  std::vector<int32_t> parent;
  std::vector<int32_t> child0;  // first of 8 consecutive children, -1 for a leaf
  std::vector<int64_t> pbeg, pend;  // point range in morton-sorted order (msort)

  // points
  std::vector<uint64_t> key;     // full-depth morton key per original point
  std::vector<int64_t> msort;    // original indices sorted by (key, index)
  std::vector<int32_t> point_leaf;  // original index -> leaf box
  std::vector<int64_t> order;    // tree order: position -> original index
  std::vector<int64_t> rank;     // original index -> tree position

  // (level, coords) -> box id; one map per level keyed by morton code
  std::vector<std::unordered_map<uint64_t, int32_t>> lookup;

  void build(const double* xyz, int64_t n, int leaf_size);

  int64_t nboxes() const { return (int64_t)level.size(); }
  bool is_leaf(int b) const { return child0[b] < 0; }
  int64_t npts(int b) const { return pend[b] - pbeg[b]; }
  double box_side(int b) const { return side / double(int64_t(1) << level[b]); }
  void box_centre(int b, double c[3]) const {
    double h = box_side(b);
    c[0] = root_lo[0] + (cx[b] + 0.5) * h;
    c[1] = root_lo[1] + (cy[b] + 0.5) * h;
    c[2] = root_lo[2] + (cz[b] + 0.5) * h;
  }
  // deepest existing box containing level-`lev` cell (x,y,z); -1 if outside the root
  int containing(int lev, int64_t x, int64_t y, int64_t z) const;
  int find(int lev, int64_t x, int64_t y, int64_t z) const;
  // first tree position of a box's points (boxes are contiguous in tree order)
  int64_t first_pos(int b) const;

 private:
  int new_box(int lev, int x, int y, int z, int par, int64_t b, int64_t e);
  void split(int b);
  void balance();
  void finish();
};

}  // namespace fmmlu
