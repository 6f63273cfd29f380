"""Pins for oracle/geometry.py: the tree and the cluster lists (Section 4.2,
table of cluster lists) against brute-force geometric definitions."""
import itertools

import numpy as np
import pytest

import workloads
from oracle.geometry import Tree, demorton, depth_for, morton


def test_depth_matches_mean_occupancy_reading():
    # kappa = smallest k >= 2 with leaf * 4^k >= N
    assert depth_for(2048, 32) == 3
    assert depth_for(65536, 64) == 5
    assert depth_for(1 << 20, 64) == 7
    assert depth_for(100, 64) == 2
    for n, s in [(5000, 32), (70000, 64), (12345, 16)]:
        k = depth_for(n, s)
        assert s * 4 ** k >= n and (k == 2 or s * 4 ** (k - 1) < n)


def test_morton_roundtrip_and_children_are_quadrants():
    for key in range(4 ** 4):
        ix, iy = demorton(key)
        assert morton(ix, iy) == key
        for c in range(4):
            cx, cy = demorton(4 * key + c)
            assert (cx >> 1, cy >> 1) == (ix, iy)
            assert (cx & 1, cy & 1) == (c & 1, c >> 1)


def _box_closed(k, m):
    ix, iy = demorton(m)
    w = 1.0 / (1 << k)
    return ix * w, (ix + 1) * w, iy * w, (iy + 1) * w


def _touch(k, a, b):
    ax0, ax1, ay0, ay1 = _box_closed(k, a)
    bx0, bx1, by0, by1 = _box_closed(k, b)
    eps = 1e-12
    return ax0 <= bx1 + eps and bx0 <= ax1 + eps and ay0 <= by1 + eps and by0 <= ay1 + eps


@pytest.mark.parametrize("k", [2, 3, 4])
def test_neighbours_and_interaction_lists_brute_force(k):
    T = Tree(workloads.uniform(64, 5), 4)
    for i in range(4 ** k):
        nbr = {j for j in range(4 ** k) if _touch(k, i, j)}
        assert set(T.neighbours(k, i)) == nbr
        # well separated: parents touch, the boxes themselves do not
        il = {j for j in range(4 ** k) if _touch(k - 1, i >> 2, j >> 2) and not _touch(k, i, j)}
        assert set(T.interaction_list(k, i)) == il
        ix, iy = demorton(i)
        if k >= 3 and 2 <= ix < (1 << k) - 2 and 2 <= iy < (1 << k) - 2:
            assert len(il) == 27 and len(nbr) == 9


def test_colour_batches_have_disjoint_neighbourhoods():
    T = Tree(workloads.uniform(64, 5), 4)
    for k in (3, 4):
        batches = T.elimination_order(k)
        assert sorted(itertools.chain(*batches)) == list(range(4 ** k))
        for b in batches:
            seen = set()
            for i in b:
                nb = set(T.neighbours(k, i))
                assert not (seen & nb)
                seen |= nb
        # every 3x3 window holds each colour exactly once
        n = 1 << k
        for x0 in range(n - 2):
            for y0 in range(n - 2):
                cols = {Tree.colour(morton(x, y)) for x in range(x0, x0 + 3) for y in range(y0, y0 + 3)}
                assert cols == set(range(9))


def test_point_order_and_leaf_membership():
    pts = workloads.uniform(3000, 11)
    T = Tree(pts, 32)
    assert sorted(T.perm.tolist()) == list(range(3000))
    nb = 1 << T.kappa
    for m in range(4 ** T.kappa):
        ix, iy = demorton(m)
        sub = T.points[T.leaf_start[m]:T.leaf_end[m]]
        assert np.all(sub[:, 0] >= ix / nb) and np.all(sub[:, 0] <= (ix + 1) / nb)
        assert np.all(sub[:, 1] >= iy / nb) and np.all(sub[:, 1] <= (iy + 1) / nb)
        idx = T.perm[T.leaf_start[m]:T.leaf_end[m]]
        assert np.all(np.diff(idx) > 0)  # stable: original order inside a leaf
    assert T.leaf_end[-1] == 3000


def test_jittered_grid_c2_has_64_points_per_leaf():
    pts = workloads.jittered_grid(65536, 1002)
    T = Tree(pts, 64)
    cnt = T.leaf_end - T.leaf_start
    assert T.kappa == 5 and cnt.min() == 64 and cnt.max() == 64
