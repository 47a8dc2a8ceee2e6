"""GPU parity of the spatial-median kd-tree (pg_kdtree_build_spatial) against
the oracle's: every node (cut value and dimension, children, leaf-order
range, depth) and the leaf-order row permutation identical; k-NN (queries,
all points, graph) and range search on it exact against the definitions."""
import numpy as np
import pytest

import oracle
from paper_2207_01834_amd import datagen
from parity import assert_float_close, assert_int_equal, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pg(dev):
    import paper_2207_01834_amd._binding as b
    b.lib()
    return b


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(*ts):
    import torch
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ts]


def check_tree(pg, dev, pts, leaf, rule="cycle", space="cell"):
    t = pg.kdtree_build(to_dev(pts, dev), leaf=leaf, split="spatial", dim_rule=rule, space=space)
    o = oracle.spatial_tree(pts, leaf=leaf, rule=rule, space=space)
    g = t.nodes()
    assert t.levels == o.depth, "depth differs"
    assert len(g["dim"]) == o.nodes, "node count differs"
    for key in ("dim", "child", "lo", "hi", "level"):
        assert np.array_equal(g[key], getattr(o, key)), f"node {key} differs"
    assert np.array_equal(g["split"].astype(np.float64), o.split), "cut values differ"
    assert np.array_equal(g["perm"].astype(np.int64), o.perm), "leaf-order rows differ"
    # leaf offsets: the leaves' ranges in leaf order
    loff = t.offsets()
    leaves = np.nonzero(g["child"] < 0)[0]
    assert len(loff) == len(leaves) + 1 and loff[0] == 0 and loff[-1] == len(pts)
    assert np.all(np.diff(loff) >= 0)
    assert np.array_equal(np.sort(g["lo"][leaves]), loff[:-1])
    return t


def leaf_sizes(t):
    g = t.nodes()
    lv = g["child"] < 0
    return g["hi"][lv] - g["lo"][lv]


def check_knn(t, pts, q, k, dev):
    if q is None:
        gi, gd = host(*t.knn_all(k))
        q = pts
    else:
        gi, gd = host(*t.knn(to_dev(q, dev), k))
    oi, od = oracle.knn_brute(pts, q, k, nthreads=8)
    if pts.dtype == np.int32:
        assert_int_equal(gi, gd, oi, od)
    else:
        assert_float_close(gi, gd, oi, od, pts, q)


@pytest.mark.parametrize("n,d,leaf,dtype,span", [
    (20_000, 2, 16, np.int32, 1 << 20), (9_000, 3, 8, np.float32, 0), (5_000, 5, 16, np.int32, 1 << 12),
    (3_000, 1, 4, np.int32, 100), (2_000, 8, 2, np.float32, 0), (4_000, 3, 1, np.int32, 6),
])
def test_spatial_tree_and_knn(pg, dev, n, d, leaf, dtype, span):
    say(f"spatial n={n} d={d} leaf={leaf} {np.dtype(dtype).name}")
    rng = np.random.default_rng(n + d + leaf)
    if dtype == np.int32:
        pts = rng.integers(-span // 2, span // 2 + 1, (n, d)).astype(np.int32)
    else:
        pts = (rng.standard_normal((n, d)) ** 3).astype(np.float32)  # skewed: uneven leaves
    t = check_tree(pg, dev, pts, leaf)
    check_knn(t, pts, None, 10, dev)
    q = pts[rng.integers(0, n, 5_000)] + (1 if dtype == np.int32 else np.float32(0.01))
    check_knn(t, pts, q.astype(dtype), 7, dev)
    gi, gd = host(*t.knn_graph(5))
    oi, od = oracle.knn_graph_brute(pts, 5, nthreads=8)
    if dtype == np.int32:
        assert_int_equal(gi, gd, oi, od)
    else:
        assert_float_close(gi, gd, oi, od, pts, pts)


def test_spatial_clustered_and_duplicates(pg, dev):
    f, q = datagen.clustered(30_000, 5, seed=3, n_queries=2_000, query_seed=33)
    t = check_tree(pg, dev, f, 16)
    assert leaf_sizes(t).max() <= 16  # split down to the leaf size
    check_knn(t, f, q, 5, dev)
    same = np.full((500, 2), 3, dtype=np.int32)
    t = check_tree(pg, dev, same, 4)
    check_knn(t, same, None, 3, dev)


def test_spatial_small_and_empty(pg, dev):
    for n in (0, 1, 2, 5):
        pts = np.arange(2 * n, dtype=np.int32).reshape(n, 2)
        t = check_tree(pg, dev, pts, 1)
        if n:
            check_knn(t, pts, None, 3, dev)


def test_spatial_range(pg, dev):
    pts = datagen.uniform_int(20_000, 2, seed=5, bits=12)
    t = pg.kdtree_build(to_dev(pts, dev), leaf=16, split="spatial")
    boxes = datagen.range_boxes(pts, 300, seed=6, m=3_000)
    off, rows = t.range_search(to_dev(boxes, dev))
    off, rows = host(off, rows)
    oc, oo, oi = oracle.range_brute(pts, boxes)
    assert np.array_equal(off, oo)
    for i in range(0, 3_000, 7):
        assert np.array_equal(np.sort(rows[off[i]:off[i + 1]].astype(np.int64)), oi[oo[i]:oo[i + 1]])


def test_spatial_full_size(pg, dev):
    """The headline points (10M 3-D int uniform, leaf 16) with spatial-median
    splits: the whole tree against the oracle's, sampled all-points rows."""
    pts = datagen.uniform_int(10_000_000, 3, seed=2)
    say("spatial 10M: build")
    t = check_tree(pg, dev, pts, 16)
    gi, gd = host(*t.knn_all(10))
    rows = np.random.default_rng(4).choice(len(pts), 300, replace=False)
    oi, od = oracle.knn_brute(pts, pts[rows], 10, nthreads=16)
    assert_int_equal(gi[rows], gd[rows], oi, od)


@pytest.mark.parametrize("n,d,leaf,dtype", [(20_000, 2, 16, np.int32), (9_000, 3, 8, np.float32),
                                            (6_000, 5, 4, np.int32), (3_000, 3, 1, np.float32)])
def test_spatial_widest_rule(pg, dev, n, d, leaf, dtype):
    # stretched boxes, so the widest side differs from the level's dimension
    rng = np.random.default_rng(n + d)
    scale = np.array([1.0, 0.05, 0.4, 2.0, 0.01][:d])
    if dtype == np.int32:
        pts = (rng.random((n, d)) * scale * 100_000).astype(np.int32)
    else:
        pts = ((rng.standard_normal((n, d)) ** 3) * scale).astype(np.float32)
    say(f"spatial widest n={n} d={d} leaf={leaf} {np.dtype(dtype).name}")
    t = check_tree(pg, dev, pts, leaf, rule="widest")
    dims = t.nodes()["dim"]
    assert len(set(dims[dims >= 0].tolist())) > 1
    check_knn(t, pts, None, 8, dev)
    q = pts[rng.integers(0, n, 5_000)]
    check_knn(t, pts, q, 5, dev)
    gi, gd = host(*t.knn_graph(4))
    oi, od = oracle.knn_graph_brute(pts, 4, nthreads=8)
    if dtype == np.int32:
        assert_int_equal(gi, gd, oi, od)
    else:
        assert_float_close(gi, gd, oi, od, pts, pts)
    boxes = datagen.range_boxes(pts, float(np.ptp(pts, axis=0).max()) * 0.05 if dtype == np.float32
                                else int(np.ptp(pts, axis=0).max() * 0.05), seed=3, m=2_000)
    off, rows = t.range_search(to_dev(boxes, dev))
    off, rows = host(off, rows)
    oc, oo, oi = oracle.range_brute(pts, boxes)
    assert np.array_equal(off, oo)
    for i in range(0, 2_000, 11):
        assert np.array_equal(np.sort(rows[off[i]:off[i + 1]].astype(np.int64)), oi[oo[i]:oo[i + 1]])


# --- nodes cutting the bounding box of their own points ----------------------

@pytest.mark.parametrize("n,d,leaf,dtype,rule", [
    (20_000, 2, 16, np.int32, "cycle"), (9_000, 3, 8, np.float32, "cycle"),
    (5_000, 5, 16, np.int32, "widest"), (3_000, 1, 4, np.int32, "cycle"),
    (2_000, 8, 2, np.float32, "widest"), (4_000, 3, 1, np.int32, "widest"),
])
def test_point_box_tree_queries(pg, dev, n, d, leaf, dtype, rule):
    say(f"point-box n={n} d={d} leaf={leaf} {np.dtype(dtype).name} {rule}")
    rng = np.random.default_rng(7 * n + d)
    if dtype == np.int32:
        pts = rng.integers(-3000, 3000, (n, d)).astype(np.int32)
        pts[: n // 3] = 100_000 + rng.integers(0, 40, (n // 3, d))  # a far, dense cluster
        pts[::7] = pts[3]  # duplicates
    else:
        pts = (rng.standard_normal((n, d)) ** 3).astype(np.float32)
        pts[: n // 3] = (5.0 + 1e-3 * rng.random((n // 3, d))).astype(np.float32)
    pts = pts[rng.permutation(n)]
    t = check_tree(pg, dev, pts, leaf, rule=rule, space="points")
    check_knn(t, pts, None, 9, dev)
    q = pts[rng.integers(0, n, 5_000)]
    check_knn(t, pts, q, 4, dev)
    gi, gd = host(*t.knn_graph(5))
    oi, od = oracle.knn_graph_brute(pts, 5, nthreads=8)
    if dtype == np.int32:
        assert_int_equal(gi, gd, oi, od)
    else:
        assert_float_close(gi, gd, oi, od, pts, pts)
    half = 50 if dtype == np.int32 else 0.05
    boxes = datagen.range_boxes(pts, half, seed=9, m=2_000)
    off, rows = t.range_search(to_dev(boxes, dev))
    off, rows = host(off, rows)
    oc, oo, oi = oracle.range_brute(pts, boxes)
    assert np.array_equal(off, oo)
    for i in range(0, 2_000, 13):
        assert np.array_equal(np.sort(rows[off[i]:off[i + 1]].astype(np.int64)), oi[oo[i]:oo[i + 1]])


def test_point_box_small_empty_and_same(pg, dev):
    for n in (0, 1, 2, 5, 33):
        pts = (np.arange(2 * n, dtype=np.int32) ** 2).reshape(n, 2)
        t = check_tree(pg, dev, pts, 1, space="points")
        if n:
            check_knn(t, pts, None, 3, dev)
    same = np.full((500, 3), -7, dtype=np.int32)
    t = check_tree(pg, dev, same, 4, rule="widest", space="points")
    check_knn(t, same, None, 3, dev)


@pytest.mark.parametrize("space", ["points", "cell"])
def test_clustered_full_size(pg, dev, space):
    """The 5-D clustered workload (10M float32 points, 1,000 clusters, 1M
    queries): the whole tree against the oracle's, every leaf at most 16
    points, every query against the oracle's search."""
    pts, q = datagen.clustered(10_000_000, 5, seed=3, n_queries=1_000_000, query_seed=33)
    say(f"clustered 10M, {space} boxes: build")
    t = check_tree(pg, dev, pts, 16, space=space)
    assert leaf_sizes(t).max() <= 16
    gi, gd = host(*t.knn(to_dev(q, dev), 5))
    del t
    oi, od, _ = oracle.KdTree(pts, leaf=16).knn(q, 5, nthreads=16)
    assert_float_close(gi, gd, oi, od, pts, q)
