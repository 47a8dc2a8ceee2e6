"""Pins for the oracle's static kd-tree (object-median splits, Appendix C /
Algorithm 1 read as: dimension = level mod d, split rank
floor((2j+1)n/2^(l+1)) under (coordinate, index), leaves at depth L)."""
import numpy as np
import pytest

import oracle
from paper_2207_01834_amd import datagen


def _node(n, l, j):
    return (j * n) >> l


def check_tree(points, leaf):
    n, d = points.shape
    t = oracle.KdTree(points, leaf=leaf)
    L = t.levels
    splits, perm = t.export()
    # (I3) depth: ceil(n/2^L) <= leaf and (L == 0 or ceil(n/2^(L-1)) > leaf)
    assert -(-n // (1 << L)) <= leaf
    if L > 0:
        assert -(-n // (1 << (L - 1))) > leaf
    # (I2) every row appears exactly once
    assert np.array_equal(np.sort(perm), np.arange(n))
    # leaf sizes in {floor(n/2^L), ceil(n/2^L)}
    sizes = np.diff([_node(n, L, j) for j in range((1 << L) + 1)])
    assert set(sizes.tolist()) <= {n >> L, -(-n // (1 << L))}
    for l in range(L):
        c = l % d
        for j in range(1 << l):
            lo, hi = _node(n, l, j), _node(n, l, j + 1)
            mid = _node(n, l + 1, 2 * j + 1)
            left, right = perm[lo:mid], perm[mid:hi]
            s = splits[(1 << l) + j - 1]
            # (I1) the split separates: left coords <= s <= right coords
            if len(left):
                assert points[left, c].max() <= s
            if len(right):
                assert points[right, c].min() == s
            # (I4) rank split under (coordinate, index): every left key is
            # below every right key, so the left set is the mid-lo smallest
            if len(left) and len(right):
                lk = max(zip(points[left, c].tolist(), left.tolist()))
                rk = min(zip(points[right, c].tolist(), right.tolist()))
                assert lk < rk
    return t


@pytest.mark.parametrize("n,d,leaf", [(0, 2, 16), (1, 3, 16), (17, 2, 1), (100, 3, 4),
                                      (1000, 2, 16), (2049, 5, 16), (777, 8, 3), (64, 1, 64)])
def test_tree_invariants_uniform(n, d, leaf):
    check_tree(datagen.uniform_int(n, d, seed=n + d), leaf)


def test_tree_invariants_duplicates_and_floats():
    g = np.random.default_rng(9)
    check_tree(g.integers(0, 3, size=(500, 3)).astype(np.int32), 5)
    check_tree(np.full((129, 2), 4, dtype=np.int32), 8)
    check_tree((np.floor(g.random((600, 2)) * 4) / 4).astype(np.float32), 7)
    check_tree(g.random((1000, 5)).astype(np.float32), 16)


def test_tree_equals_sort_based_construction():
    # The median-partition step reduces to a library sort: sort every node
    # by (coordinate, index) and cut at the split position.
    g = np.random.default_rng(4)
    pts = g.integers(0, 20, size=(1500, 3)).astype(np.int32)
    n, d, leaf = len(pts), 3, 6
    t = oracle.KdTree(pts, leaf=leaf)
    splits, perm = t.export()
    L = t.levels
    ref = np.arange(n)
    ref_splits = np.zeros((1 << L) - 1)
    for l in range(L):
        c = l % d
        for j in range(1 << l):
            lo, hi = _node(n, l, j), _node(n, l, j + 1)
            seg = ref[lo:hi]
            order = np.lexsort((seg, pts[seg, c]))
            ref[lo:hi] = seg[order]
            mid = _node(n, l + 1, 2 * j + 1)
            ref_splits[(1 << l) + j - 1] = pts[ref[mid], c]
    assert np.array_equal(splits, ref_splits)
    for j in range(1 << L):
        lo, hi = _node(n, L, j), _node(n, L, j + 1)
        assert set(perm[lo:hi].tolist()) == set(ref[lo:hi].tolist())


def test_cfg1_depth_and_leaves():
    # 2-D, n = 10,000, leaf 16: L = 10, 1,024 leaves of 9 or 10 points.
    assert oracle.tree_depth(10_000, 16) == 10
    assert oracle.tree_depth(10_000_000, 16) == 20
    pts = datagen.uniform_int(10_000, 2, seed=1)
    t = check_tree(pts, 16)
    assert t.levels == 10


# --- spatial-median tree (cell halving) -------------------------------------

def test_spatial_hand_worked_int_and_float():
    # 1-D int 0..9: root cell [0, 9] cut at floor(10/2) = 5; [0, 4] at
    # floor(5/2) = 2; [5, 9] at floor(15/2) = 7.  Depth 2 for leaf 3.
    pts = np.arange(10, dtype=np.int32).reshape(-1, 1)
    L, s, _, perm, loff = oracle.spatial_tree(pts, leaf=3)
    assert L == 2 and s[1:].tolist() == [5, 2, 7]
    assert loff.tolist() == [0, 2, 5, 7, 10] and perm.tolist() == list(range(10))
    # 1-D float {0, .25, .5, .75, 1}: [0, 1] at .5; [0, .5] at .25; [.5, 1] at .75
    f = np.array([1.0, 0.5, 0.0, 0.75, 0.25], dtype=np.float32).reshape(-1, 1)
    L, s, _, perm, loff = oracle.spatial_tree(f, leaf=2)
    assert L == 2 and s[1:].tolist() == [0.5, 0.25, 0.75]
    # stable: rows 0 (1.0) and 3 (0.75) keep their input order in the last leaf
    assert loff.tolist() == [0, 1, 2, 3, 5] and perm.tolist() == [2, 4, 1, 0, 3]


def test_spatial_full_grid_is_morton_order():
    # all of {0..15}^2 with one point per leaf: the cells are dyadic, so the
    # leaf of (x, y) interleaves the bits of x and y (x first, high bits first)
    k = 4
    xs, ys = np.meshgrid(np.arange(1 << k), np.arange(1 << k), indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)
    rng = np.random.default_rng(0)
    pts = pts[rng.permutation(len(pts))]
    L, s, _, perm, loff = oracle.spatial_tree(pts, leaf=1)
    assert L == 2 * k and np.all(np.diff(loff) == 1)

    def morton(x, y):
        m = 0
        for b in range(k - 1, -1, -1):
            m = (m << 2) | (((x >> b) & 1) << 1) | ((y >> b) & 1)
        return m

    want = np.argsort([morton(int(x), int(y)) for x, y in pts])
    assert perm.tolist() == want.tolist()


def test_spatial_identical_points_go_right():
    pts = np.full((37, 3), 5, dtype=np.int32)
    L, s, _, perm, loff = oracle.spatial_tree(pts, leaf=4)
    sizes = np.diff(loff)
    assert sizes[-1] == 37 and sizes[:-1].sum() == 0 and perm.tolist() == list(range(37))


@pytest.mark.parametrize("d,leaf,dtype", [(2, 4, np.int32), (3, 8, np.float32), (5, 2, np.int32)])
def test_spatial_invariants(d, leaf, dtype):
    rng = np.random.default_rng(d * 10 + leaf)
    n = 3000
    if dtype == np.int32:
        pts = rng.integers(-500, 500, (n, d)).astype(np.int32)
        pts[::5] = pts[7]
    else:
        pts = (rng.standard_normal((n, d)) ** 3).astype(np.float32)
    L, s, _, perm, loff = oracle.spatial_tree(pts, leaf=leaf)
    assert L == oracle.tree_depth(n, leaf)
    assert sorted(perm.tolist()) == list(range(n))
    leaf_of = np.repeat(np.arange(1 << L), np.diff(loff))
    # rows ascending inside every leaf (each side keeps the parent's order)
    for j in range(1 << L):
        rows = perm[loff[j]:loff[j + 1]]
        assert np.all(np.diff(rows) > 0)
    # every internal node separates: left coordinates < split <= right ones
    P = pts[perm].astype(np.float64)
    for h in range(1, 1 << L):
        l = h.bit_length() - 1
        j = h - (1 << l)
        c = l % d
        span = 1 << (L - l)
        lo, mid, hi = loff[j * span], loff[j * span + span // 2], loff[(j + 1) * span]
        assert np.all(P[lo:mid, c] < s[h]) and np.all(P[mid:hi, c] >= s[h])


def test_spatial_widest_rule_hand_worked():
    # cell 0..31 x 0..15: x is widest -> cut at 16; each half is 16 x 16, a
    # tie -> x again (the lowest dimension): 8 and 24; then y (8 x 16) at 8
    xs, ys = np.meshgrid(np.arange(32), np.arange(16), indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)
    L, s, dims, perm, loff = oracle.spatial_tree(pts, leaf=64, rule="widest")
    assert L == 3
    assert dims[1:4].tolist() == [0, 0, 0] and s[1:4].tolist() == [16, 8, 24]
    assert dims[4:8].tolist() == [1, 1, 1, 1] and s[4:8].tolist() == [8, 8, 8, 8]
    assert np.all(np.diff(loff) == 64)
    # the cyclic rule cuts y at the second level instead
    L, s, dims, perm, loff = oracle.spatial_tree(pts, leaf=64, rule="cycle")
    assert dims[1:4].tolist() == [0, 1, 1] and s[1:4].tolist() == [16, 8, 8]


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_spatial_widest_invariants(dtype):
    rng = np.random.default_rng(9)
    n, d, leaf = 4000, 3, 8
    scale = np.array([1000.0, 30.0, 200.0])
    pts = (rng.random((n, d)) * scale).astype(dtype)
    L, s, dims, perm, loff = oracle.spatial_tree(pts, leaf=leaf, rule="widest")
    assert dims[1] == 0  # the root's widest side
    P = pts[perm].astype(np.float64)
    for h in range(1, 1 << L):
        l = h.bit_length() - 1
        j = h - (1 << l)
        c = dims[h]
        span = 1 << (L - l)
        lo, mid, hi = loff[j * span], loff[j * span + span // 2], loff[(j + 1) * span]
        assert np.all(P[lo:mid, c] < s[h]) and np.all(P[mid:hi, c] >= s[h])
    for j in range(1 << L):
        assert np.all(np.diff(perm[loff[j]:loff[j + 1]]) > 0)


# --- spatial-median tree, each node cutting the bounding box of its points ---

def test_spatial_point_box_hand_worked():
    # 1-D int {100, 2, 0, 1}, leaf 1 (depth 2).  Point boxes: root [0, 100]
    # cut at floor(101/2) = 50; left {2, 0, 1}: box [0, 2] cut at
    # floor(3/2) = 1 -> {0} | {2, 1}; right {100}: box [100, 100] cut at
    # 100 -> {} | {100}.
    pts = np.array([[100], [2], [0], [1]], dtype=np.int32)
    L, s, dims, perm, loff = oracle.spatial_tree(pts, leaf=1, space="points")
    assert L == 2 and s[1:].tolist() == [50, 1, 100] and dims[1:].tolist() == [0, 0, 0]
    assert loff.tolist() == [0, 1, 3, 3, 4] and perm.tolist() == [2, 1, 3, 0]
    # cell halving on the same points: [0, 49] cut at 25, [50, 100] at 75
    L, s, _, perm, loff = oracle.spatial_tree(pts, leaf=1, space="cell")
    assert s[1:].tolist() == [50, 25, 75] and loff.tolist() == [0, 3, 3, 3, 4]
    # float {0, .25, .5, 4}: [0, 4] at 2; [0, .5] at .25; [4, 4] at 4
    f = np.array([[4.0], [0.5], [0.0], [0.25]], dtype=np.float32)
    L, s, _, perm, loff = oracle.spatial_tree(f, leaf=1, space="points")
    assert s[1:].tolist() == [2.0, 0.25, 4.0]
    assert loff.tolist() == [0, 1, 3, 3, 4] and perm.tolist() == [2, 1, 3, 0]


def test_spatial_point_box_empty_node():
    # {0..6, 1000}, leaf 1 (depth 3): the root cuts [0, 1000] at 500; the
    # right node {1000} cuts [1000, 1000] at 1000, so its left child (node 6,
    # an internal node) is empty and takes split 0
    pts = np.array([[v] for v in (0, 1, 2, 3, 4, 5, 6, 1000)], dtype=np.int32)
    L, s, dims, perm, loff = oracle.spatial_tree(pts, leaf=1, space="points")
    assert L == 3 and s[1] == 500 and s[3] == 1000 and s[6] == 0
    assert np.diff(loff).tolist()[4:] == [0, 0, 0, 1]
    # 2-D: an empty node takes dimension l mod d, or 0 under the widest rule
    p2 = np.array([[0, 0], [1, 5], [2, 1], [3, 3], [4, 2], [5, 6], [6, 4], [1000, 9]], dtype=np.int32)
    for rule in ("cycle", "widest"):
        L, s, dims, perm, loff = oracle.spatial_tree(p2, leaf=1, rule=rule, space="points")
        for h in range(1, 1 << L):
            l = h.bit_length() - 1
            span = 1 << (L - l)
            j = h - (1 << l)
            if loff[j * span] == loff[(j + 1) * span]:
                assert s[h] == 0 and dims[h] == (l % 2 if rule == "cycle" else 0)


@pytest.mark.parametrize("rule,dtype", [("cycle", np.int32), ("widest", np.int32),
                                        ("cycle", np.float32), ("widest", np.float32)])
def test_spatial_point_box_invariants(rule, dtype):
    # a dense cluster beside a sparse background: every split lies inside its
    # node's point box and separates it; the widest rule takes that box's
    # widest side; once the cluster's node holds only cluster points, cutting
    # point boxes spreads it over many leaves, while cell halving keeps it in
    # one leaf (its cells stay far wider than the cluster)
    rng = np.random.default_rng(31)
    n, d, leaf = 4000, 3, 8
    if dtype == np.int32:
        bg = rng.integers(0, 1 << 19, (n // 4, d))
        cl = 1_000_000 + rng.integers(0, 64, (n - n // 4, d))
    else:
        bg = 0.5 * rng.random((n // 4, d))
        cl = 0.95 + 1e-4 * rng.random((n - n // 4, d))
    pts = np.concatenate([bg, cl]).astype(dtype)[rng.permutation(n)]
    L, s, dims, perm, loff = oracle.spatial_tree(pts, leaf=leaf, rule=rule, space="points")
    assert sorted(perm.tolist()) == list(range(n))
    P = pts[perm].astype(np.float64)
    for h in range(1, 1 << L):
        l = h.bit_length() - 1
        j = h - (1 << l)
        span = 1 << (L - l)
        lo, mid, hi = loff[j * span], loff[j * span + span // 2], loff[(j + 1) * span]
        if lo == hi:
            continue
        box_lo, box_hi = P[lo:hi].min(axis=0), P[lo:hi].max(axis=0)
        c = dims[h]
        if rule == "widest":
            assert c == int(np.argmax(box_hi - box_lo))
        else:
            assert c == l % d
        assert box_lo[c] <= s[h] <= box_hi[c]
        assert np.all(P[lo:mid, c] < s[h]) and np.all(P[mid:hi, c] >= s[h])
    for j in range(1 << L):
        assert np.all(np.diff(perm[loff[j]:loff[j + 1]]) > 0)
    cell = oracle.spatial_tree(pts, leaf=leaf, rule=rule, space="cell")[4]
    assert 8 * np.diff(loff).max() < np.diff(cell).max()
