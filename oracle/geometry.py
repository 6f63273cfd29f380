"""Uniform quadtree, Z order and cluster lists.

Paper: Section 4.2 (uniform 2^d tree; table "Different lists associated with
cluster i at level k": N_i = neighbours including self, I_i = children of the
parent's neighbours that are well separated); Section 2.2 figure of the 2D
FMM matrix (Morton / Z ordering).

Readings taken where the paper is silent:
* depth: kappa = max(2, ceil(log4(N / leaf_size))), i.e. the mean leaf
  occupancy is at most leaf_size;
* a point's box index is floor((x - lo) / size * 2^k) clamped to 2^k - 1;
* points are ordered by (leaf Morton key, original index);
* elimination order inside a level: nine colours 3*(ix mod 3) + (iy mod 3),
  colour by colour, Morton order inside a colour.
"""
from __future__ import annotations

import numpy as np


def depth_for(n: int, leaf_size: int) -> int:
    k = 2
    while leaf_size * 4 ** k < n:
        k += 1
    return k


def morton(ix: int, iy: int) -> int:
    key = 0
    b = 0
    while (ix >> b) or (iy >> b):
        key |= ((ix >> b) & 1) << (2 * b)
        key |= ((iy >> b) & 1) << (2 * b + 1)
        b += 1
    return key


def demorton(key: int) -> tuple[int, int]:
    ix = iy = 0
    b = 0
    while key >> (2 * b):
        ix |= ((key >> (2 * b)) & 1) << b
        iy |= ((key >> (2 * b + 1)) & 1) << b
        b += 1
    return ix, iy


class Tree:
    """Uniform quadtree over the square [lo, lo + size]^2 with depth kappa.

    Clusters at level k are indexed by their Morton key in [0, 4^k).  The
    children of cluster m are 4m + c, c = 0..3 with (dx, dy) = (c & 1, c >> 1).
    """

    def __init__(self, points: np.ndarray, leaf_size: int, lo=(0.0, 0.0), size=1.0):
        pts = np.asarray(points, dtype=np.float64)
        self.N = pts.shape[0]
        self.kappa = depth_for(self.N, leaf_size)
        self.lo = (float(lo[0]), float(lo[1]))
        self.size = float(size)
        nb = 1 << self.kappa
        bx = np.minimum(np.floor((pts[:, 0] - self.lo[0]) / self.size * nb), nb - 1).astype(np.int64)
        by = np.minimum(np.floor((pts[:, 1] - self.lo[1]) / self.size * nb), nb - 1).astype(np.int64)
        keys = np.array([morton(int(a), int(b)) for a, b in zip(bx, by)], dtype=np.int64)
        # stable sort by (key, original index)
        self.perm = np.lexsort((np.arange(self.N), keys))
        self.points = pts[self.perm]
        sk = keys[self.perm]
        nleaf = 4 ** self.kappa
        self.leaf_start = np.searchsorted(sk, np.arange(nleaf), side="left")
        self.leaf_end = np.searchsorted(sk, np.arange(nleaf), side="right")

    # ---- geometry of boxes -------------------------------------------------
    def box(self, k: int, m: int):
        """Centre and half-width of cluster m at level k."""
        ix, iy = demorton(m)
        w = self.size / (1 << k)
        return (self.lo[0] + (ix + 0.5) * w, self.lo[1] + (iy + 0.5) * w), 0.5 * w

    def leaf_points(self, m: int) -> np.ndarray:
        return self.points[self.leaf_start[m]:self.leaf_end[m]]

    # ---- lists ----------------------------------------------------------------
    def neighbours(self, k: int, m: int) -> list[int]:
        """N_i: clusters at Chebyshev box distance <= 1, including i itself."""
        ix, iy = demorton(m)
        n = 1 << k
        out = []
        for jx in range(ix - 1, ix + 2):
            for jy in range(iy - 1, iy + 2):
                if 0 <= jx < n and 0 <= jy < n:
                    out.append(morton(jx, jy))
        return sorted(out)

    def interaction_list(self, k: int, m: int) -> list[int]:
        """I_i: children of the parent's neighbours that are not neighbours of i."""
        if k < 2:
            return []
        par = m >> 2
        near = set(self.neighbours(k, m))
        out = []
        for pn in self.neighbours(k - 1, par):
            for c in range(4):
                ch = 4 * pn + c
                if ch not in near:
                    out.append(ch)
        return sorted(out)

    @staticmethod
    def adjacent(a: int, b: int) -> bool:
        ax, ay = demorton(a)
        bx, by = demorton(b)
        return max(abs(ax - bx), abs(ay - by)) <= 1

    @staticmethod
    def colour(m: int) -> int:
        ix, iy = demorton(m)
        return 3 * (ix % 3) + (iy % 3)

    def elimination_order(self, k: int) -> list[list[int]]:
        """Nine batches (one per colour), Morton order inside each batch."""
        batches = [[] for _ in range(9)]
        for m in range(4 ** k):
            batches[self.colour(m)].append(m)
        return batches
