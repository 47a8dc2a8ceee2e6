"""Pins for the oracle's well-separated pair decomposition (the kd-tree's
WSPD, Section 2's second module, read as Callahan and Kosaraju's recursive
pairing with ball separation of bounding boxes): hand-worked pair sets on a
line, and, by brute force over the points, that every pair of distinct
points is covered by exactly one pair and that every pair's point sets are
separated (their closest points at least s times half the larger
diameter apart, which ball separation implies)."""
import itertools

import numpy as np
import pytest

import oracle


def test_hand_worked_line():
    # points 0, 1, 2, 3 (leaf 1): the root's children {0,1} (node 2) and
    # {2,3} (node 3) have radius 1/2 and centres 2 apart: separated for
    # s = 2 ((s + 2) r = 2), so the pairs are (2,3), (4,5), (6,7)
    t = oracle.KdTree(np.array([[0], [1], [2], [3]], np.int32), leaf=1)
    assert t.wspd(2.0).tolist() == [[2, 3], [4, 5], [6, 7]]
    # s = 2.01: (2,3) is not; equal radii split the first node; {0} vs
    # {2,3} (centre gap 2.5 >= 4.01 / 2) is separated; {1} vs {2,3} (gap
    # 1.5) is not and splits the larger node {2,3}; single points always are
    assert t.wspd(2.01).tolist() == [[4, 3], [5, 6], [5, 7], [4, 5], [6, 7]]
    # two points: one pair; one point or none: no pairs
    assert oracle.KdTree(np.array([[5, 1], [5, 1]], np.int32), leaf=1).wspd(1.0).tolist() == [[2, 3]]
    assert len(oracle.KdTree(np.zeros((1, 2), np.int32), leaf=1).wspd(1.0)) == 0
    assert len(oracle.KdTree(np.zeros((0, 2), np.int32), leaf=1).wspd(1.0)) == 0


def test_bad_arguments():
    t = oracle.KdTree(np.arange(20, dtype=np.int32).reshape(10, 2), leaf=2)
    with pytest.raises(ValueError):
        t.wspd(2.0)  # leaf size above 1
    t = oracle.KdTree(np.arange(20, dtype=np.int32).reshape(10, 2), leaf=1)
    for s in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(ValueError):
            t.wspd(s)


def check_wspd(pts, s):
    n = len(pts)
    t = oracle.KdTree(pts, leaf=1)
    pairs = t.wspd(s)
    _, perm = t.export()
    P = pts.astype(np.float64)
    cover = np.zeros((n, n), dtype=np.int64)
    for a, b in pairs:
        A = perm[slice(*t.node_range(a))]
        B = perm[slice(*t.node_range(b))]
        assert len(A) and len(B)
        cover[np.ix_(A, B)] += 1
        cover[np.ix_(B, A)] += 1
        # separation: closest points at least s * (larger diameter) / 2 apart
        dmin = np.sqrt(((P[A][:, None, :] - P[B][None, :, :]) ** 2).sum(-1)).min()
        diam = max(np.sqrt(((P[X][:, None, :] - P[X][None, :, :]) ** 2).sum(-1)).max() for X in (A, B))
        assert dmin >= s * diam / 2 * (1 - 1e-12), (a, b, dmin, diam)
    off = ~np.eye(n, dtype=bool)
    assert np.all(cover[off] == 1), "a pair of points is covered other than once"
    assert np.all(np.diag(cover) == 0)
    return pairs


@pytest.mark.parametrize("n,d,dtype,s", [(2, 2, np.int32, 2.0), (3, 1, np.int32, 2.0),
                                         (17, 2, np.int32, 2.0), (120, 2, np.int32, 1.0),
                                         (150, 3, np.float32, 2.0), (200, 2, np.float32, 4.0),
                                         (90, 5, np.int32, 2.0), (64, 2, np.int32, 8.0)])
def test_cover_once_and_separated(n, d, dtype, s):
    g = np.random.default_rng(n + d)
    if dtype == np.int32:
        pts = g.integers(0, 50, (n, d)).astype(np.int32)  # duplicates
    else:
        pts = (g.standard_normal((n, d)) ** 3).astype(np.float32)
    pairs = check_wspd(pts, s)
    assert len(pairs) >= n - 1  # at least one pair per internal node with points


def test_grid_and_identical_points():
    grid = np.array(list(itertools.product(range(8), range(8))), dtype=np.int32)
    check_wspd(grid, 2.0)
    same = np.full((40, 3), 7, dtype=np.int32)
    pairs = check_wspd(same, 2.0)
    # identical points: every pair is separated at once (radius 0), so the
    # pairs are the children of the internal nodes that hold points
    assert len(pairs) == 39
