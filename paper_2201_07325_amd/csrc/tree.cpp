// Level-restricted adaptive octree on the host.
//
// Points are quantised once onto a 2^21 grid per axis inside the root cube and sorted by
// their full-depth Morton key; every box at every level is then a contiguous range of
// that order, so splitting a box is a partition of its range by the next three key bits.
// The level restriction is enforced finest level first: each leaf looks at the 26 cells
// around it at its own level and splits any leaf found there that is more than one level
// coarser. Splits only create coarser-than-current leaves, which are visited later, so
// one pass suffices; every split is forced, so the result is the unique minimal
// balanced refinement.
#include "tree.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>
#include <vector>

#include "common.hpp"

namespace fmmlu {

static inline uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffff;
  x = (x | (x << 32)) & 0x1f00000000ffffULL;
  x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
  x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
  x = (x | (x << 2)) & 0x1249249249249249ULL;
  return x;
}

// fn(lo, hi) over [0, n) in contiguous chunks on up to 8 threads (inline when small)
template <class F>
static void chunked(int64_t n, int64_t grain, F&& fn) {
  const int64_t nt = std::max<int64_t>(1, std::min<int64_t>({8, (int64_t)std::thread::hardware_concurrency(), n / grain}));
  if (nt <= 1) {
    fn(int64_t(0), n);
    return;
  }
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::thread> th;
  for (int64_t t = 1; t < nt; ++t)
    th.emplace_back([&, t] { fn(t * chunk, std::min(n, (t + 1) * chunk)); });
  fn(int64_t(0), std::min(n, chunk));
  for (auto& x : th) x.join();
}

uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

int Octree::new_box(int lev, int x, int y, int z, int par, int64_t b, int64_t e) {
  int id = (int)level.size();
  level.push_back((int8_t)lev);
  cx.push_back(x);
  cy.push_back(y);
  cz.push_back(z);
  parent.push_back(par);
  child0.push_back(-1);
  pbeg.push_back(b);
  pend.push_back(e);
  if ((int)lookup.size() <= lev) lookup.resize(lev + 1);
  lookup[lev][morton3(x, y, z)] = id;
  return id;
}

void Octree::split(int b) {
  int lev = level[b];
  int shift = 3 * (kDepth - lev - 1);
  int64_t lo = pbeg[b], hi = pend[b];
  int first = (int)level.size();
  int bx = cx[b], by = cy[b], bz = cz[b];
  int64_t cur = lo;
  for (int o = 0; o < 8; ++o) {
    // points of octant o form the next run of the sorted range
    int64_t e = cur;
    while (e < hi && (int)((key[msort[e]] >> shift) & 7) == o) ++e;
    new_box(lev + 1, 2 * bx + (o & 1), 2 * by + ((o >> 1) & 1), 2 * bz + ((o >> 2) & 1), b, cur, e);
    cur = e;
  }
  child0[b] = first;
}

int Octree::find(int lev, int64_t x, int64_t y, int64_t z) const {
  if (lev >= (int)lookup.size()) return -1;
  auto it = lookup[lev].find(morton3((uint32_t)x, (uint32_t)y, (uint32_t)z));
  return it == lookup[lev].end() ? -1 : it->second;
}

int Octree::containing(int lev, int64_t x, int64_t y, int64_t z) const {
  int64_t lim = int64_t(1) << lev;
  if (x < 0 || y < 0 || z < 0 || x >= lim || y >= lim || z >= lim) return -1;
  for (int l = lev; l >= 0; --l) {
    int sh = lev - l;
    int b = find(l, x >> sh, y >> sh, z >> sh);
    if (b >= 0) return b;
  }
  return -1;
}

void Octree::balance() {
  int maxlev = 0;
  for (auto l : level) maxlev = std::max<int>(maxlev, l);
  for (int lev = maxlev; lev >= 2; --lev) {
    std::vector<int> leaves;
    for (int b = 0; b < (int)level.size(); ++b)
      if (level[b] == lev && child0[b] < 0) leaves.push_back(b);
    for (int b : leaves) {
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy && !dz) continue;
            int64_t x = cx[b] + dx, y = cy[b] + dy, z = cz[b] + dz;
            for (;;) {
              int a = containing(lev, x, y, z);
              if (a < 0) break;
              if (child0[a] < 0 && level[a] < lev - 1)
                split(a);
              else
                break;
            }
          }
    }
  }
}

int64_t Octree::first_pos(int b) const {
  // all points of box b are contiguous in tree order; empty boxes have none
  if (pend[b] == pbeg[b]) return -1;
  int64_t best = INT64_MAX;
  for (int64_t i = pbeg[b]; i < pend[b]; ++i) best = std::min(best, rank[msort[i]]);
  return best;
}

void Octree::finish() {
  nlevels = 0;
  for (auto l : level) nlevels = std::max<int>(nlevels, l + 1);
  point_leaf.assign(n, -1);
  for (int b = 0; b < (int)level.size(); ++b)
    if (child0[b] < 0)
      for (int64_t i = pbeg[b]; i < pend[b]; ++i) point_leaf[msort[i]] = b;
  // tree order: leaves by the Morton key of their lower corner at full depth, then
  // original index. Leaves are disjoint ranges of msort in Morton order, so re-sorting
  // each leaf's range by original index gives the tree order.
  order.resize(n);
  std::vector<int> leaves;
  for (int b = 0; b < (int)level.size(); ++b)
    if (child0[b] < 0 && pend[b] > pbeg[b]) leaves.push_back(b);
  std::sort(leaves.begin(), leaves.end(), [&](int a, int b) { return pbeg[a] < pbeg[b]; });
  // leaf l's run starts at the sum of the earlier leaves' sizes; runs are independent
  std::vector<int64_t> start(leaves.size() + 1, 0);
  for (size_t l = 0; l < leaves.size(); ++l) start[l + 1] = start[l] + (pend[leaves[l]] - pbeg[leaves[l]]);
  chunked((int64_t)leaves.size(), 256, [&](int64_t lo, int64_t hi) {
    for (int64_t l = lo; l < hi; ++l) {
      const int b = leaves[l];
      int64_t pos = start[l];
      for (int64_t i = pbeg[b]; i < pend[b]; ++i) order[pos++] = msort[i];
      std::sort(order.begin() + start[l], order.begin() + pos);
    }
  });
  rank.resize(n);
  chunked(n, 8192, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) rank[order[i]] = i;
  });
}

void Octree::build(const double* xyz, int64_t n_, int leaf_size_) {
  n = n_;
  leaf_size = leaf_size_;
  const double* X[3] = {xyz, xyz + n, xyz + 2 * n};
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = hi[a] = X[a][0];
    for (int64_t i = 1; i < n; ++i) {
      lo[a] = std::min(lo[a], X[a][i]);
      hi[a] = std::max(hi[a], X[a][i]);
    }
  }
  double ext = 0.0;
  for (int a = 0; a < 3; ++a) ext = std::max(ext, hi[a] - lo[a]);
  side = ext * (1.0 + 1e-12);
  if (side == 0.0) side = 1.0;
  for (int a = 0; a < 3; ++a) root_lo[a] = 0.5 * (lo[a] + hi[a]) - 0.5 * side;
  const double scale = double(int64_t(1) << kDepth);
  const int64_t qmax = (int64_t(1) << kDepth) - 1;
  key.resize(n);
  chunked(n, 8192, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      uint32_t q[3];
      for (int a = 0; a < 3; ++a) {
        volatile double t = (X[a][i] - root_lo[a]) / side;  // no contraction: match IEEE order
        double u = std::floor(t * scale);
        int64_t v = (int64_t)u;
        q[a] = (uint32_t)std::min<int64_t>(std::max<int64_t>(v, 0), qmax);
      }
      key[i] = morton3(q[0], q[1], q[2]);
    }
  });
  // order by (key, index): least-significant-digit radix sort of (key, index) pairs, stable
  // and started in index order, so equal keys keep increasing indices
  {
    std::vector<std::pair<uint64_t, int64_t>> a((size_t)n), b((size_t)n);
    for (int64_t i = 0; i < n; ++i) a[i] = {key[i], i};
    for (int sh = 0; sh < 3 * kDepth; sh += 8) {
      size_t cnt[257] = {0};
      for (const auto& e : a) ++cnt[((e.first >> sh) & 255) + 1];
      if (cnt[((a[0].first >> sh) & 255) + 1] == (size_t)n) continue;  // one digit value: order unchanged
      for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
      for (const auto& e : a) b[cnt[(e.first >> sh) & 255]++] = e;
      a.swap(b);
    }
    msort.resize(n);
    for (int64_t i = 0; i < n; ++i) msort[i] = a[i].second;
  }
  level.clear(); cx.clear(); cy.clear(); cz.clear(); parent.clear(); child0.clear();
  pbeg.clear(); pend.clear(); lookup.clear();
  new_box(0, 0, 0, 0, -1, 0, n);
  std::vector<int> stack{0};
  while (!stack.empty()) {
    int b = stack.back();
    stack.pop_back();
    if (npts(b) > leaf_size && level[b] < kDepth) {
      split(b);
      for (int o = 0; o < 8; ++o) stack.push_back(child0[b] + o);
    }
  }
  balance();
  finish();
}

}  // namespace fmmlu
