"""Pins for the CPU oracle's k-NN parts (brute force = the definition, and
the kd-tree search of Appendix C), checked against closed forms, an
independent library (SciPy's kd-tree), invariants and brute force."""
import numpy as np
import pytest

import oracle
from paper_2207_01834_amd import datagen

INT64_MAX = np.iinfo(np.int64).max


def test_pythagorean_closed_form():
    # Points at integer multiples of the (3,4,5) and (5,12,13) triples:
    # squared distances 25 a^2 and 169 b^2 are known without the formula.
    pts = np.array([[0, 0], [3, 4], [6, 8], [5, 12], [-3, -4], [0, 0], [-5, 12]], dtype=np.int32)
    q = np.array([[0, 0]], dtype=np.int32)
    ids, dist = oracle.knn_brute(pts, q, 7)
    # D: id0 0, id5 0 (tie -> smaller id first), id1 25, id4 25, id2 100, id3 169, id6 169
    assert ids.tolist() == [[0, 5, 1, 4, 2, 3, 6]]
    assert dist.tolist() == [[0, 0, 25, 25, 100, 169, 169]]
    # from (3,4): id1 at 0; ids 0, 2 and 5 all at 25 (the smaller ids win)
    ids, dist = oracle.knn_brute(pts, np.array([[3, 4]], dtype=np.int32), 3)
    assert ids.tolist() == [[1, 0, 2]] and dist.tolist() == [[0, 25, 25]]


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_lattice_shell_multiplicities(d):
    # Integer lattice {0..6}^d with spacing s: an interior point has exactly
    # 2d neighbours at D = s^2 and 2d(d-1) at D = 2 s^2.
    s = 7
    axes = [np.arange(7) * s] * d
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, d).astype(np.int32)
    q = np.full((1, d), 3 * s, dtype=np.int32)
    k = 1 + 2 * d + 2 * d * (d - 1)
    ids, dist = oracle.knn_brute(grid, q, k)
    dist = dist[0]
    assert dist[0] == 0
    assert np.count_nonzero(dist == s * s) == 2 * d
    assert np.count_nonzero(dist == 2 * s * s) == 2 * d * (d - 1)
    # the nearest point is the query itself, its id is its row in the grid
    assert ids[0, 0] == int(np.nonzero((grid == q).all(axis=1))[0][0])
    # within each shell ids ascend (ties broken by the smaller id)
    for shell in (s * s, 2 * s * s):
        sel = ids[0][dist == shell]
        assert np.all(np.diff(sel) > 0)


def test_against_scipy_kdtree():
    spatial = pytest.importorskip("scipy.spatial")
    g = np.random.default_rng(11)
    for d in (1, 2, 3, 5, 8):
        pts = g.integers(0, 1 << 9, size=(700, d)).astype(np.int32)
        qs = g.integers(0, 1 << 9, size=(60, d)).astype(np.int32)
        k = 9
        ids, dist = oracle.knn_brute(pts, qs, k)
        sd, _ = spatial.cKDTree(pts.astype(np.float64)).query(qs.astype(np.float64), k=k)
        sd = np.rint(np.asarray(sd).reshape(len(qs), k) ** 2).astype(np.int64)
        assert np.array_equal(np.sort(sd, axis=1), dist)
        # every returned id really is at the returned distance
        diff = qs[:, None, :].astype(np.int64) - pts[ids].astype(np.int64)
        assert np.array_equal(np.sum(diff * diff, axis=2), dist)


def test_metamorphic_translation_permutation_prefix():
    g = np.random.default_rng(5)
    pts = g.integers(0, 50, size=(400, 3)).astype(np.int32)  # many ties
    qs = g.integers(0, 50, size=(50, 3)).astype(np.int32)
    ids, dist = oracle.knn_brute(pts, qs, 12)
    # translation
    t = np.array([1000, -77, 3], dtype=np.int32)
    ids2, dist2 = oracle.knn_brute(pts + t, qs + t, 12)
    assert np.array_equal(ids, ids2) and np.array_equal(dist, dist2)
    # row permutation with ids carried along
    perm = g.permutation(len(pts))
    ids3, dist3 = oracle.knn_brute(pts[perm], qs, 12, ids=perm.astype(np.int64))
    assert np.array_equal(ids, ids3) and np.array_equal(dist, dist3)
    # prefix: the k=5 result is the first 5 of the k=12 result
    ids4, dist4 = oracle.knn_brute(pts, qs, 5)
    assert np.array_equal(ids[:, :5], ids4) and np.array_equal(dist[:, :5], dist4)
    # scaling by 3 multiplies distances by 9
    ids5, dist5 = oracle.knn_brute(pts * 3, qs * 3, 12)
    assert np.array_equal(ids, ids5) and np.array_equal(dist * 9, dist5)


def test_int_float_cross_pin():
    # x / 2^20 is exact in float32 and its FP64 squared distances are the
    # integer ones times 2^-40 exactly.
    pts = datagen.uniform_int(3000, 3, seed=7)
    qs = pts[:200]
    ids_i, d_i = oracle.knn_brute(pts, qs, 10)
    f = datagen.int_to_unit_float(pts)
    ids_f, d_f = oracle.knn_brute(f, f[:200], 10)
    assert np.array_equal(ids_i, ids_f)
    assert np.array_equal(d_i.astype(np.float64) * 2.0 ** -40, d_f)


def test_padding_when_fewer_points():
    pts = np.array([[1, 1], [2, 2]], dtype=np.int32)
    ids, dist = oracle.knn_brute(pts, pts, 4)
    assert ids.tolist() == [[0, 1, -1, -1], [1, 0, -1, -1]]
    assert dist[0, 2] == INT64_MAX and dist[1, 3] == INT64_MAX
    f = pts.astype(np.float32)
    ids, dist = oracle.knn_brute(f, f, 3)
    assert ids[0, 2] == -1 and np.isinf(dist[0, 2])
    ids, dist = oracle.knn_brute(np.zeros((0, 2), np.int32), pts, 2)
    assert (ids == -1).all()


def _cases():
    g = np.random.default_rng(2024)
    out = []
    for trial in range(40):
        d = int(g.integers(1, 9))
        n = int(g.choice([0, 1, 2, 5, 17, 100, 999, 2500, 5000]))
        k = int(g.integers(1, min(n + 4, 40) + 1))
        leaf = int(g.choice([1, 2, 3, 8, 16, 64]))
        kind = trial % 4
        if kind == 0:
            p = g.integers(0, 1 << 20, size=(n, d)).astype(np.int32)
        elif kind == 1:
            p = g.integers(-3, 4, size=(n, d)).astype(np.int32)  # heavy duplicates
        elif kind == 2:
            p = g.random((n, d)).astype(np.float32)
        else:
            p = (np.floor(g.random((n, d)) * 8) / 8).astype(np.float32)  # float ties
        out.append((p, k, leaf))
    return out


@pytest.mark.parametrize("case", range(40))
def test_kd_knn_equals_brute(case):
    p, k, leaf = _cases()[case]
    q = p[: min(len(p), 300)]
    if len(q) == 0:
        q = np.zeros((3, p.shape[1]), dtype=p.dtype)
    t = oracle.KdTree(p, leaf=leaf)
    ids, dist, cnt = t.knn(q, k)
    ids_b, dist_b = oracle.knn_brute(p, q, k)
    assert np.array_equal(ids, ids_b)
    assert np.array_equal(dist, dist_b)


def test_kd_knn_visits_far_fewer_points_than_brute():
    p = datagen.uniform_int(100_000, 3, seed=3)
    t = oracle.KdTree(p, leaf=16)
    _, _, cnt = t.knn(p[:500], 10)
    per_q = cnt[2] / 500
    assert per_q < 1000  # empirically logarithmic (Appendix C), far below n


def test_all_identical_points():
    p = np.full((300, 3), 5, dtype=np.int32)
    t = oracle.KdTree(p, leaf=4)
    ids, dist, _ = t.knn(p[:10], 7)
    assert (dist == 0).all()
    assert np.array_equal(ids, np.tile(np.arange(7), (10, 1)))


def _graph_loops(pts, k):
    # pure-Python definition on tiny inputs: sort the other points by (D, j)
    n = len(pts)
    rows_i, rows_d = [], []
    for i in range(n):
        keys = sorted((int(((pts[i].astype(np.int64) - pts[j]) ** 2).sum()), j)
                      for j in range(n) if j != i)[:k]
        keys += [(INT64_MAX, -1)] * (k - len(keys))
        rows_i.append([j for _, j in keys])
        rows_d.append([dd for dd, _ in keys])
    return np.array(rows_i), np.array(rows_d)


@pytest.mark.parametrize("n,k,span", [(1, 3, 5), (2, 3, 5), (7, 3, 2), (40, 5, 3), (60, 4, 100)])
def test_knn_graph_excludes_only_self(n, k, span):
    # small coordinate spans force many identical points: an identical point
    # is a neighbour at distance 0, the point itself never is
    rng = np.random.default_rng(n * 31 + k)
    pts = rng.integers(0, span, (n, 2)).astype(np.int32)
    gi, gd = oracle.knn_graph_brute(pts, k)
    wi, wd = _graph_loops(pts, k)
    assert gi.tolist() == wi.tolist() and gd.tolist() == wd.tolist()
    assert not np.any(gi == np.arange(n)[:, None])


def test_knn_graph_many_duplicates_drop_last():
    # 12 identical points, k = 10: for row 11 the k+1 nearest (ids 0..10)
    # do not include itself; the graph row is ids 0..9
    pts = np.zeros((12, 3), dtype=np.int32)
    gi, gd = oracle.knn_graph_brute(pts, 10)
    assert gi[11].tolist() == list(range(10)) and gd[11].tolist() == [0] * 10
    assert gi[0].tolist() == list(range(1, 11))


# --- the search's visit counters, on trees small enough to walk by hand ------
# (internal nodes entered, leaves whose points were offered, points offered).
# Tree over the 1-D points 0..7 with leaf 2: the root splits at the value of
# rank 4 (4), level 1 at ranks 2 and 6 (values 2 and 6), leaves {0,1} {2,3}
# {4,5} {6,7}.

def _line_tree():
    pts = np.arange(8, dtype=np.int32).reshape(-1, 1)
    t = oracle.KdTree(pts, leaf=2)
    assert t.export()[0].tolist() == [4, 2, 6]
    return t


def test_visit_counters_hand_worked_1d():
    t = _line_tree()
    # q = 3, k = 3: root (internal 1) -> node [0,4) (internal 2) -> leaf
    # {2,3} (2 points); fewer than k, so the sibling leaf {0,1} is added
    # whole (2 more); back at the root the 3rd key is (4, id 1) and the far
    # node [4,8) has box [4, 7], lower bound 1 <= 4: entered (internal 3),
    # its near leaf {4,5} added (6 points); the 3rd key is now (1, id 4) and
    # leaf {6,7} (lower bound 9) is pruned.
    ids, dist, c = t.knn(np.array([[3]], np.int32), 3)
    assert ids.tolist() == [[3, 2, 4]] and dist.tolist() == [[0, 1, 1]]
    assert c.tolist() == [3, 3, 6]
    # q = 4, k = 2: root -> [4,8) -> leaf {4,5}; the 2nd key (1, id 5) prunes
    # {6,7} (lower bound 4); back at the root the box [0, 3] has lower bound
    # 1, not above 1: entered (internal 3), leaf {2,3} offered; the 2nd key
    # becomes (1, id 3) and {0,1} (lower bound 9) is pruned.
    ids, dist, c = t.knn(np.array([[4]], np.int32), 2)
    assert ids.tolist() == [[4, 3]] and dist.tolist() == [[0, 1]]
    assert c.tolist() == [3, 2, 4]
    # q = 3, k = 6: too few candidates after each near subtree, so every
    # sibling subtree is added whole: 2 internal nodes, 4 leaves, 8 points
    ids, dist, c = t.knn(np.array([[3]], np.int32), 6)
    assert ids.tolist() == [[3, 2, 4, 1, 5, 0]] and c.tolist() == [2, 4, 8]
    # counters sum over queries; q = 4, k = 3 mirrors q = 3 (root -> [4,8)
    # -> {4,5}, sibling {6,7} added, [0,4) entered, {2,3} offered, {0,1}
    # pruned): 3, 3, 6 each
    _, _, c = t.knn(np.array([[3], [4]], np.int32), 3)
    assert c.tolist() == [6, 6, 12]


def test_visit_counters_hand_worked_contained_subtree():
    # 2-D, leaf 1: rows (0,0) (0,100) (1,50) (1,51).  The root splits x at
    # rank 2 (x = 1); the left node splits y at its rank-1 point (y = 100),
    # the right node at y = 51.  Query (0, 100), k = 2: root -> left node ->
    # leaf {(0,100)} (D 0); the sibling leaf {(0,0)} is added (D 10000);
    # back at the root the right node's box x [1,1], y [50,51] lies within
    # the 2nd distance (its farthest corner is at 1 + 50^2 = 2501 <= 10000),
    # so it is added whole without entering it: 2 internal nodes, 4 leaves,
    # 4 points.
    pts = np.array([[0, 0], [0, 100], [1, 50], [1, 51]], dtype=np.int32)
    t = oracle.KdTree(pts, leaf=1)
    assert t.export()[0].tolist() == [1, 100, 51]
    ids, dist, c = t.knn(np.array([[0, 100]], np.int32), 2)
    assert ids.tolist() == [[1, 3]] and dist.tolist() == [[0, 2402]]
    assert c.tolist() == [2, 4, 4]


def test_kd_knn_threaded_chunks_change_nothing():
    # the query-parallel form runs the same serial search on static chunks
    g = np.random.default_rng(31)
    pts = g.integers(0, 300, size=(5000, 3)).astype(np.int32)
    q = g.integers(0, 300, size=(777, 3)).astype(np.int32)
    t = oracle.KdTree(pts, leaf=8)
    a = t.knn(q, 9)
    for th in (2, 5, 16):
        b = t.knn(q, 9, nthreads=th)
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
