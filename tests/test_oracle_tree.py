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


# --- spatial-median tree (split until a node holds at most `leaf` points) ---

def _sp(pts, leaf, rule="cycle", space="cell"):
    return oracle.spatial_tree(np.asarray(pts), leaf=leaf, rule=rule, space=space)


def _leaf_rows(t):
    return [t.perm[t.lo[u]:t.hi[u]].tolist() for u in t.leaves]


def test_spatial_hand_worked_1d_int():
    # 0..9, leaf 3: root cell [0, 9] cut at floor(10/2) = 5; left {0..4} (5 > 3
    # points) cell [0, 4] cut at floor(5/2) = 2; right {5..9} cell [5, 9] cut at
    # floor(15/2) = 7; the four children hold 2, 3, 2, 3 points: leaves.
    t = _sp(np.arange(10, dtype=np.int32).reshape(-1, 1), 3)
    assert t.nodes == 7 and t.depth == 3
    assert t.split[:3].tolist() == [5, 2, 7] and t.dim[:3].tolist() == [0, 0, 0]
    assert t.child.tolist() == [1, 3, 5, -1, -1, -1, -1]
    assert t.lo.tolist() == [0, 0, 5, 0, 2, 5, 7] and t.hi.tolist() == [10, 5, 10, 2, 5, 7, 10]
    assert t.level.tolist() == [0, 1, 1, 2, 2, 2, 2]
    assert t.perm.tolist() == list(range(10))


def test_spatial_hand_worked_variable_depth_cell_and_box():
    # {0, 1000..1004} in the input order below, leaf 2.  Cell halving: the
    # root [0, 1004] cuts at 502: {0} | {1000..1004}; the right cell [502,
    # 1004] then cuts at 753, 879, 942, 973, 989, 997 with an empty left child
    # each time; [997, 1004] cuts at 1001: {1000} | {1001..1004}; [1001, 1004]
    # cuts at 1003: {1001, 1002} | {1003, 1004}.
    vals = [1003, 0, 1001, 1000, 1004, 1002]
    pts = np.array(vals, dtype=np.int32).reshape(-1, 1)
    t = _sp(pts, 2)
    inner = t.child >= 0
    assert t.split[inner].tolist() == [502, 753, 879, 942, 973, 989, 997, 1001, 1003]
    assert t.depth == 10
    assert [[vals[r] for r in rows] for rows in _leaf_rows(t)] == \
        [[0]] + [[]] * 6 + [[1000], [1001, 1002], [1003, 1004]]
    assert t.leaf_sizes().max() <= 2
    # point boxes: the root box [0, 1004] cuts at 502; {1000..1004} has box
    # [1000, 1004], cut at floor(2005/2) = 1002: {1001, 1000} | {1003, 1004,
    # 1002} (input order kept); the latter, box [1002, 1004], cuts at 1003:
    # {1002} | {1003, 1004}.
    t = _sp(pts, 2, space="points")
    assert t.split[t.child >= 0].tolist() == [502, 1002, 1003]
    assert [[vals[r] for r in rows] for rows in _leaf_rows(t)] == \
        [[0], [1001, 1000], [1002], [1003, 1004]]
    assert t.depth == 4


def test_spatial_hand_worked_float():
    # {1, .5, 0, .75, .25}, leaf 2: cell [0, 1] cuts at .5: {0, .25} | {1, .5,
    # .75}; the right cell [.5, 1] cuts at .75: {.5} | {1, .75}.  The left
    # cell of a float cut ends at the float just below the cut.
    f = np.array([1.0, 0.5, 0.0, 0.75, 0.25], dtype=np.float32).reshape(-1, 1)
    t = _sp(f, 2)
    assert t.split[t.child >= 0].tolist() == [0.5, 0.75]
    assert _leaf_rows(t) == [[2, 4], [1], [0, 3]]
    # two adjacent floats: the nearest float to their midpoint is the lower
    # one (ties to even), so the cut moves up to the upper one
    one = np.float32(1.0)
    up = np.nextafter(one, np.float32(2.0))
    g = np.array([up, one, up, one, one, up], dtype=np.float32).reshape(-1, 1)
    t = _sp(g, 2)
    assert t.nodes == 3 and t.split[0] == float(up)
    assert _leaf_rows(t) == [[1, 3, 4], [0, 2, 5]]


def test_spatial_identical_points_form_one_leaf():
    # more identical points than `leaf`: no cut can separate them
    t = _sp(np.full((37, 3), 5, dtype=np.int32), 4)
    assert t.nodes == 1 and t.child[0] == -1 and t.hi[0] == 37
    # beside one other point: the root cuts [5, 9] at 7 (dimension 0); the
    # 37 identical points then form one leaf
    pts = np.full((38, 3), 5, dtype=np.int32)
    pts[17] = 9
    for space in ("cell", "points"):
        t = _sp(pts, 4, space=space)
        assert t.nodes == 3 and t.split[0] == 7
        assert _leaf_rows(t) == [[r for r in range(38) if r != 17], [17]]


def test_spatial_full_grid_is_morton_order():
    # all of {0..15}^2 with one point per leaf: the cells are dyadic, so the
    # leaves, all at depth 8, come in the order that interleaves the bits of
    # x and y (x first, high bits first)
    k = 4
    xs, ys = np.meshgrid(np.arange(1 << k), np.arange(1 << k), indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)
    rng = np.random.default_rng(0)
    pts = pts[rng.permutation(len(pts))]
    t = _sp(pts, 1)
    assert t.depth == 2 * k + 1 and t.nodes == 2 * len(pts) - 1
    assert np.all(t.level[t.leaves] == 2 * k) and np.all(t.leaf_sizes() == 1)

    def morton(x, y):
        m = 0
        for b in range(k - 1, -1, -1):
            m = (m << 2) | (((x >> b) & 1) << 1) | ((y >> b) & 1)
        return m

    want = np.argsort([morton(int(x), int(y)) for x, y in pts])
    assert t.perm.tolist() == want.tolist()


def test_spatial_widest_rule_hand_worked():
    # cell 0..31 x 0..15, leaf 64: x is widest -> cut at 16; each half is
    # 16 x 16, a tie -> x again (the lowest dimension): 8 and 24; then y
    # (8 x 16) at 8; 64 points per node: leaves
    xs, ys = np.meshgrid(np.arange(32), np.arange(16), indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)
    t = _sp(pts, 64, rule="widest")
    assert t.nodes == 15
    assert t.dim[:7].tolist() == [0, 0, 0, 1, 1, 1, 1]
    assert t.split[:7].tolist() == [16, 8, 24, 8, 8, 8, 8]
    assert np.all(t.leaf_sizes() == 64)
    # the cyclic rule cuts y at the second level instead
    t = _sp(pts, 64, rule="cycle")
    assert t.dim[:3].tolist() == [0, 1, 1] and t.split[:3].tolist() == [16, 8, 8]


def _check_structure(t, pts, leaf, rule, space):
    """Invariants of a spatial tree: ranges nest and partition, every cut
    separates its node, lies in its space and takes the rule's dimension,
    leaves hold at most `leaf` points unless identical, rows keep their
    order inside each leaf (stable partitions)."""
    n, d = pts.shape
    P = pts[t.perm].astype(np.float64)
    assert sorted(t.perm.tolist()) == list(range(n))
    assert t.lo[0] == 0 and t.hi[0] == n
    for u in range(t.nodes):
        lo, hi = t.lo[u], t.hi[u]
        if t.child[u] < 0:
            box = P[lo:hi]
            if hi - lo > leaf:
                assert np.all(box == box[0]), f"leaf {u} of {hi - lo} non-identical points"
            assert np.all(np.diff(t.perm[lo:hi]) > 0)
            continue
        a = t.child[u]
        assert t.lo[a] == lo and t.hi[a] == t.lo[a + 1] and t.hi[a + 1] == hi
        assert t.level[a] == t.level[a + 1] == t.level[u] + 1
        c, s = t.dim[u], t.split[u]
        assert np.all(P[lo:t.hi[a], c] < s) and np.all(P[t.lo[a + 1]:hi, c] >= s)
        blo, bhi = P[lo:hi].min(axis=0), P[lo:hi].max(axis=0)
        if space == "points":
            assert blo[c] < s <= bhi[c] or blo[c] == bhi[c] == s
            if rule == "widest":
                assert c == int(np.argmax(bhi - blo))
        if rule == "cycle":
            assert c == t.level[u] % d
    # breadth-first numbering: levels non-decreasing, leaf order within a level
    assert np.all(np.diff(t.level) >= 0)
    for lv in range(t.depth):
        sel = np.nonzero(t.level == lv)[0]
        assert np.all(np.diff(t.lo[sel]) >= 0)


@pytest.mark.parametrize("d,leaf,dtype,rule,space", [
    (2, 4, np.int32, "cycle", "cell"), (3, 8, np.float32, "cycle", "cell"),
    (5, 2, np.int32, "widest", "cell"), (3, 8, np.float32, "widest", "points"),
    (2, 1, np.int32, "cycle", "points"), (4, 16, np.float32, "cycle", "points")])
def test_spatial_invariants(d, leaf, dtype, rule, space):
    rng = np.random.default_rng(d * 10 + leaf)
    n = 3000
    if dtype == np.int32:
        pts = rng.integers(-500, 500, (n, d)).astype(np.int32)
        pts[::5] = pts[7]          # heavy duplicates
    else:
        pts = (rng.standard_normal((n, d)) ** 3).astype(np.float32)
        pts[::7] = pts[3]
    t = _sp(pts, leaf, rule, space)
    _check_structure(t, pts, leaf, rule, space)


@pytest.mark.parametrize("space", ["cell", "points"])
def test_spatial_dense_cluster_is_resolved(space):
    # a dense cluster beside a sparse background: the cluster is cut until
    # every leaf holds at most `leaf` points (the fixed-depth reading had left
    # it in one leaf); cell halving reaches it deeper than point boxes do
    rng = np.random.default_rng(31)
    n, d, leaf = 4000, 3, 8
    bg = rng.integers(0, 1 << 19, (n // 4, d))
    cl = 1_000_000 + rng.integers(0, 4096, (n - n // 4, d))
    pts = np.concatenate([bg, cl]).astype(np.int32)[rng.permutation(n)]
    t = _sp(pts, leaf, space=space)
    _check_structure(t, pts, leaf, "cycle", space)
    assert t.leaf_sizes().max() <= leaf
    deep = _sp(pts, leaf, space="cell").depth
    assert t.depth <= deep


def test_spatial_small_and_empty():
    for n in (0, 1, 2, 16, 17):
        pts = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
        t = _sp(pts, 16)
        assert t.hi[0] == n
        assert t.nodes == (1 if n <= 16 else 3)
