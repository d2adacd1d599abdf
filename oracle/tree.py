"""Level-restricted adaptive octree (oracle; test infrastructure).

Section 4 (opening): the root is a cube C containing all points (level 0); a box at
level l is split into eight equal children while it holds more than s points; the
childless boxes are the leaves. Two leaves that share a boundary point (face, edge
or corner) must be at most one level apart; this is enforced afterwards by splitting
the coarser leaf.

Readings where the paper leaves details open:
  * Root cube: centred on the bounding box of the points, side = largest extent
    times (1 + 1e-12) (1 when all points coincide).
  * Box membership uses half-open intervals; points are first quantised to a
    2^21 grid per axis, q_a = floor((x_a - lo_a) / side * 2^21) clamped to the grid,
    and a box at level l with integer coordinates c holds the points whose q >> (21 - l)
    equals c. Children are numbered by octant o = bx + 2 by + 4 bz.
  * All eight children of a split box exist, empty ones included, and the level
    restriction applies to every leaf.
  * Tree order of the points: by the Morton key of their leaf's lower corner at full
    depth, then by original index. Every box's points are contiguous in this order.
"""
from __future__ import annotations

import numpy as np

DEPTH = 21
_OFFS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
         if (dx, dy, dz) != (0, 0, 0)]


def quantise(x):
    """Root cube and per-point integer coordinates on the 2^DEPTH grid."""
    lo = x.min(axis=1)
    hi = x.max(axis=1)
    centre = 0.5 * (lo + hi)
    side = float((hi - lo).max()) * (1.0 + 1e-12)
    if side == 0.0:
        side = 1.0
    root_lo = centre - 0.5 * side
    scale = float(1 << DEPTH)
    q = np.floor((x - root_lo[:, None]) / side * scale)
    q = np.clip(q, 0, (1 << DEPTH) - 1).astype(np.int64)
    return root_lo, side, q


def morton(ix, iy, iz):
    """Interleave the low DEPTH bits of three non-negative integers (x lowest)."""
    ix, iy, iz = (np.asarray(v, dtype=np.uint64) for v in (ix, iy, iz))
    key = np.zeros(np.broadcast(ix, iy, iz).shape, dtype=np.uint64)
    for b in range(DEPTH):
        ub = np.uint64(b)
        one = np.uint64(1)
        key |= ((ix >> ub) & one) << np.uint64(3 * b)
        key |= ((iy >> ub) & one) << np.uint64(3 * b + 1)
        key |= ((iz >> ub) & one) << np.uint64(3 * b + 2)
    return key


class Tree:
    """Boxes are stored in flat lists; box b has level[b], coord[b] = (ix, iy, iz),
    parent[b], children[b] (8 ids or None) and pts[b] (original point indices)."""

    def __init__(self, x, leaf_size=64):
        x = np.asarray(x, dtype=np.float64)
        self.n = x.shape[1]
        self.leaf_size = int(leaf_size)
        self.root_lo, self.side, self.q = quantise(x)
        self.level, self.coord, self.parent, self.children, self.pts = [], [], [], [], []
        self.lookup = {}
        self._new_box(0, (0, 0, 0), -1, np.arange(self.n))
        # 1. split while count > s (Section 4, opening)
        stack = [0]
        while stack:
            b = stack.pop()
            if self.pts[b].size > self.leaf_size and self.level[b] < DEPTH:
                stack.extend(self._split(b))
        # 2. level restriction, finest leaves first (Section 4, opening)
        self._balance()
        self._finish()

    # -- construction ---------------------------------------------------------------
    def _new_box(self, lev, c, par, pts):
        b = len(self.level)
        self.level.append(lev)
        self.coord.append(tuple(int(v) for v in c))
        self.parent.append(par)
        self.children.append(None)
        self.pts.append(pts)
        self.lookup[(lev, *self.coord[b])] = b
        return b

    def _split(self, b):
        lev = self.level[b]
        cx, cy, cz = self.coord[b]
        p = self.pts[b]
        sh = DEPTH - lev - 1
        bits = (self.q[:, p] >> sh) & 1
        octant = bits[0] + 2 * bits[1] + 4 * bits[2]
        kids = []
        for o in range(8):
            bx, by, bz = o & 1, (o >> 1) & 1, (o >> 2) & 1
            kids.append(self._new_box(lev + 1, (2 * cx + bx, 2 * cy + by, 2 * cz + bz), b,
                                      np.sort(p[octant == o])))
        self.children[b] = kids
        return kids

    def _containing(self, lev, c):
        """Deepest existing box that contains level-`lev` cell c."""
        for l2 in range(lev, -1, -1):
            sh = lev - l2
            key = (l2, c[0] >> sh, c[1] >> sh, c[2] >> sh)
            if key in self.lookup:
                return self.lookup[key]
        raise AssertionError("root must exist")

    def _balance(self):
        maxlev = max(self.level)
        for lev in range(maxlev, 1, -1):
            leaves = [b for b in range(len(self.level))
                      if self.level[b] == lev and self.children[b] is None]
            for b in leaves:
                c = self.coord[b]
                for d in _OFFS:
                    nc = (c[0] + d[0], c[1] + d[1], c[2] + d[2])
                    if min(nc) < 0 or max(nc) >= (1 << lev):
                        continue
                    while True:
                        a = self._containing(lev, nc)
                        if self.children[a] is None and self.level[a] < lev - 1:
                            self._split(a)
                        else:
                            break

    def _finish(self):
        nb = len(self.level)
        self.level = np.array(self.level, dtype=np.int64)
        self.coord = np.array(self.coord, dtype=np.int64).reshape(nb, 3)
        self.parent = np.array(self.parent, dtype=np.int64)
        self.is_leaf = np.array([c is None for c in self.children])
        self.nlevels = int(self.level.max()) + 1
        self.point_leaf = np.empty(self.n, dtype=np.int64)
        for b in np.nonzero(self.is_leaf)[0]:
            self.point_leaf[self.pts[b]] = b
        lev = self.level[self.point_leaf]
        corner = self.coord[self.point_leaf] << (DEPTH - lev)[:, None]
        key = morton(corner[:, 0], corner[:, 1], corner[:, 2])
        self.order = np.lexsort((np.arange(self.n), key))
        self.rank = np.empty(self.n, dtype=np.int64)
        self.rank[self.order] = np.arange(self.n)

    # -- queries --------------------------------------------------------------------
    def box_side(self, b):
        return self.side / (1 << int(self.level[b]))

    def box_centre(self, b):
        h = self.box_side(b)
        return self.root_lo + (self.coord[b] + 0.5) * h

    def leaves(self):
        return np.nonzero(self.is_leaf)[0]

    def ancestor(self, b, lev):
        while self.level[b] > lev:
            b = self.parent[b]
        return b

    def summary(self):
        """Sorted (level, ix, iy, iz, npoints, is_leaf) rows; implementation-independent."""
        rows = [(int(self.level[b]), *map(int, self.coord[b]), int(self.pts[b].size),
                 int(self.is_leaf[b])) for b in range(len(self.level))]
        return sorted(rows)


def touching(lev1, c1, lev2, c2):
    """True when the closed boxes (lev1, c1) and (lev2, c2) share at least one point."""
    L = max(lev1, lev2)
    s1, s2 = 1 << (L - lev1), 1 << (L - lev2)
    for a in range(3):
        lo1, hi1 = c1[a] * s1, (c1[a] + 1) * s1
        lo2, hi2 = c2[a] * s2, (c2[a] + 1) * s2
        if lo1 > hi2 or lo2 > hi1:
            return False
    return True


def linf_gap(lev, c, lev2, c2):
    """L-infinity gap between box (lev, c) and a box (lev2 <= lev, c2), in units of the
    level-`lev` box side."""
    s2 = 1 << (lev - lev2)
    g = 0
    for a in range(3):
        lo2, hi2 = c2[a] * s2, (c2[a] + 1) * s2
        g = max(g, lo2 - (c[a] + 1), c[a] - hi2)
    return max(g, 0)
