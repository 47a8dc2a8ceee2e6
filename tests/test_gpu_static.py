"""GPU parity of the static kd-tree path against the CPU oracle (through the
C ABI): tree structure, all-points and query k-NN, edge cases, full-size
sampled rows."""
import numpy as np
import pytest

import oracle
from paper_2207_01834_amd import datagen
from parity import assert_float_close, assert_int_equal, compare_tree, say

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


def run_case(pg, dev, pts, k, leaf, queries=None, check_tree=True):
    say(f"case n={len(pts)} d={pts.shape[1]} k={k} leaf={leaf} dtype={pts.dtype} queries={None if queries is None else len(queries)}")
    t = pg.kdtree_build(to_dev(pts, dev), leaf=leaf)
    if check_tree:
        compare_tree(t, pts, leaf)
    if queries is None:
        gi, gd = host(*t.knn_all(k))
        q = pts
    else:
        gi, gd = host(*t.knn(to_dev(queries, dev), k))
        q = queries
    oi, od = oracle.knn_brute(pts, q, k, nthreads=8)
    if pts.dtype == np.int32:
        assert_int_equal(gi, gd, oi, od)
    else:
        assert_float_close(gi, gd, oi, od, pts, q)
    return t


def test_cfg1_2d_all_points(pg, dev):
    pts = datagen.uniform_int(10_000, 2, seed=1)
    t = run_case(pg, dev, pts, 10, 16)
    assert t.levels == 10


def test_cfg1_float_variant_and_cross_pin(pg, dev):
    pts = datagen.uniform_int(10_000, 2, seed=1)
    f = datagen.int_to_unit_float(pts)
    run_case(pg, dev, f, 10, 16)
    # the float neighbour sets equal the int ones except fp32 near-ties
    ti = pg.kdtree_build(to_dev(pts, dev), leaf=16)
    tf = pg.kdtree_build(to_dev(f, dev), leaf=16)
    ii, di = host(*ti.knn_all(10))
    fi, fd = host(*tf.knn_all(10))
    same = (ii == fi).all(axis=1)
    assert same.mean() > 0.99
    exact = di.astype(np.float64) * 2.0 ** -40
    rel = np.abs(fd - exact) / np.where(exact == 0, 1, exact)
    assert rel.max() <= 1e-6


def _small_cases():
    g = np.random.default_rng(77)
    out = []
    ns = [0, 1, 2, 5, 63, 64, 65, 1000, 2047, 2048, 2049, 4097, 20000]
    for i in range(36):
        d = int(g.integers(1, 9))
        n = ns[i % len(ns)]
        leaf = int(g.choice([1, 2, 5, 16, 64]))
        k = int(g.choice([1, 2, 7, 10, 16, 33, 64]))
        kind = i % 4
        if kind == 0:
            p = g.integers(0, 1 << 20, size=(n, d)).astype(np.int32)
        elif kind == 1:
            p = g.integers(-4, 4, size=(n, d)).astype(np.int32)
        elif kind == 2:
            p = (g.standard_normal((n, d)) * 100).astype(np.float32)
        else:
            p = (np.floor(g.random((n, d)) * 16) / 16 - 0.5).astype(np.float32)
        qmode = i % 3  # 0: all points, 1: separate queries, 2: queries = points
        out.append((p, k, leaf, qmode, int(g.integers(0, 1 << 30))))
    return out


@pytest.mark.parametrize("case", range(36))
def test_small_random(pg, dev, case):
    p, k, leaf, qmode, seed = _small_cases()[case]
    g = np.random.default_rng(seed)
    q = None
    if qmode == 1:
        m = int(g.integers(1, 300))
        if p.dtype == np.int32:
            q = g.integers(-10, (1 << 20) + 10, size=(m, p.shape[1])).astype(np.int32)
        else:
            q = (g.standard_normal((m, p.shape[1])) * 100).astype(np.float32)
    elif qmode == 2 and len(p):
        q = p.copy()
    run_case(pg, dev, p, k, leaf, q)


def test_ties_identical_grid_planes(pg, dev):
    run_case(pg, dev, np.full((5000, 3), 7, dtype=np.int32), 10, 16)
    ax = np.arange(24, dtype=np.int32)
    grid = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3).copy()
    t = run_case(pg, dev, grid, 7, 4)
    gi, gd = host(*t.knn_all(7))
    interior = ((grid > 0) & (grid < 23)).all(axis=1)
    assert (gd[interior][:, 1:] == 1).all()  # 2d = 6 neighbours at D = 1
    g = np.random.default_rng(5)
    planes = g.choice(np.array([0, 1 << 10, 1 << 19], dtype=np.int32), size=(30000, 2))
    run_case(pg, dev, planes, 12, 8, queries=planes[:500].copy())


def test_wide_distances_exact_redo(pg, dev):
    # int32 searches order packed (distance, id) keys whose distance field
    # has 64 - ceil(log2 n) bits; queries whose k-th distance does not fit
    # are searched again with exact pairs.  Full-range coordinates make most
    # k-th distances too large, a dense core next to them mixes redone and
    # packed queries in one wave.
    g = np.random.default_rng(11)
    lo, hi = -(1 << 29), (1 << 29)
    wide = g.integers(lo, hi, size=(20000, 3)).astype(np.int32)
    run_case(pg, dev, wide, 10, 16)
    core = g.integers(0, 1 << 12, size=(15000, 3)).astype(np.int32)
    mixed = np.concatenate([core, wide[:5000]])
    g.shuffle(mixed)
    run_case(pg, dev, mixed, 10, 16)
    q = np.concatenate([g.integers(lo, hi, size=(3000, 3)), g.integers(0, 1 << 12, size=(3000, 3))]).astype(np.int32)
    run_case(pg, dev, mixed, 7, 8, queries=q, check_tree=False)
    run_case(pg, dev, g.integers(lo, hi, size=(5000, 8)).astype(np.int32), 16, 16)


def test_wide_and_middle_levels(pg, dev):
    # 1.2M points: levels 0-8 take the multi-workgroup path, level 9 the
    # one-workgroup-per-node path, the rest the LDS subtree path.
    pts = datagen.uniform_int(1_200_000, 3, seed=21)
    say("wide/middle int 1.2M")
    t = pg.kdtree_build(to_dev(pts, dev), leaf=16)
    ot = compare_tree(t, pts, 16)
    gi, gd = host(*t.knn_all(10))
    rows = np.random.default_rng(0).choice(len(pts), 3000, replace=False)
    oi, od, _ = ot.knn(pts[rows], 10)
    assert_int_equal(gi[rows], gd[rows], oi, od)
    f, q = datagen.clustered(1_200_000, 5, seed=3, n_queries=20_000, query_seed=33)
    say("wide/middle float clustered 5D 1.2M")
    t = pg.kdtree_build(to_dev(f, dev), leaf=16)
    ot = compare_tree(t, f, 16)
    gi, gd = host(*t.knn(to_dev(q, dev), 5))
    oi, od, _ = ot.knn(q, 5)
    assert_float_close(gi, gd, oi, od, f, q)


def test_full_size_cfg2(pg, dev):
    """The benchmarked configuration (3-D, n = 10M, k = 10, leaf 16, all
    points): every row against the oracle's kd-tree search, byte-identical
    for int32; the float32 variant (int / 2^20, exact) every row to the bar."""
    pts = datagen.uniform_int(10_000_000, 3, seed=2)
    say("cfg2 int 10M")
    t = pg.kdtree_build(to_dev(pts, dev), leaf=16)
    assert t.levels == 20
    gi, gd = host(*t.knn_all(10))
    del t
    say("cfg2 int 10M: oracle")
    ot = oracle.KdTree(pts, leaf=16)
    oi, od, _ = ot.knn(pts, 10, nthreads=16)
    del ot
    assert_int_equal(gi, gd, oi, od)
    int_ids = oi
    del gi, gd, od
    f = datagen.int_to_unit_float(pts)
    say("cfg2 float 10M")
    t = pg.kdtree_build(to_dev(f, dev), leaf=16)
    gi, gd = host(*t.knn_all(10))
    del t
    say("cfg2 float 10M: oracle")
    ot = oracle.KdTree(f, leaf=16)
    oi, od, _ = ot.knn(f, 10, nthreads=16)
    del ot
    assert_float_close(gi, gd, oi, od, f, f)
    # the coordinates are exact dyadics, so the FP64 oracle's rows are the
    # int rows: the float32 ids differ from them only at near-ties
    assert np.array_equal(oi, int_ids)


def test_full_size_clustered_5d(pg, dev):
    # The benchmarked 5-D clustered configuration: 10M float32 points from a
    # 1,000-cluster mixture, 1M queries from the same mixture, k = 5, leaf 16
    # (the query set is large enough to be reordered by leaf): every query.
    f, q = datagen.clustered(10_000_000, 5, seed=3, n_queries=1_000_000, query_seed=33)
    say("cfg3 clustered 5-D 10M, 1M queries")
    t = pg.kdtree_build(to_dev(f, dev), leaf=16)
    assert t.levels == 20
    gi, gd = host(*t.knn(to_dev(q, dev), 5))
    del t
    say("cfg3: oracle")
    oi, od, _ = oracle.KdTree(f, leaf=16).knn(q, 5, nthreads=16)
    assert_float_close(gi, gd, oi, od, f, q)


def test_determinism(pg, dev):
    pts = datagen.uniform_int(300_000, 3, seed=9)
    a = pg.kdtree_build(to_dev(pts, dev), leaf=16)
    b = pg.kdtree_build(to_dev(pts, dev), leaf=16)
    ai, ad = host(*a.knn_all(10))
    bi, bd = host(*b.knn_all(10))
    assert np.array_equal(ai, bi) and np.array_equal(ad, bd)
    sa, pa = a.export()
    sb, pb = b.export()
    assert np.array_equal(sa, sb) and np.array_equal(pa, pb)


def test_range_errors(pg, dev):
    bad = np.array([[0, 0], [1 << 29, 5]], dtype=np.int32)
    with pytest.raises(pg.RangeError):
        pg.kdtree_build(to_dev(bad, dev), leaf=4)
    nan = np.array([[0.0, 1.0], [np.nan, 2.0]], dtype=np.float32)
    with pytest.raises(pg.RangeError):
        pg.kdtree_build(to_dev(nan, dev), leaf=4)
    t = pg.kdtree_build(to_dev(np.zeros((4, 2), np.int32), dev), leaf=4)
    with pytest.raises(pg.RangeError):
        t.knn(to_dev(np.array([[-(1 << 29) - 1, 0]], dtype=np.int32), dev), 2)
    # -0.0 is stored as +0.0
    z = np.array([[-0.0, 1.0], [0.0, 1.0]], dtype=np.float32)
    t = pg.kdtree_build(to_dev(z, dev), leaf=1)
    gi, gd = host(*t.knn_all(2))
    assert (gd == 0).all() and gi.tolist() == [[0, 1], [0, 1]]


def graph_oracle_rows(pts, rows, k):
    """k-NN graph rows of the sampled points from the definition: the k+1
    nearest of each sampled point over all points, its own entry removed."""
    oi, od = oracle.knn_brute(pts, pts[rows], k + 1, nthreads=16)
    own = oi == rows[:, None]
    keep = ~own
    keep[own.sum(axis=1) == 0, k] = False
    return oi[keep].reshape(len(rows), k), od[keep].reshape(len(rows), k)


@pytest.mark.parametrize("n,d,k,leaf,dtype,span", [
    (1, 2, 3, 16, np.int32, 100), (2, 3, 1, 1, np.int32, 100), (5, 2, 4, 1, np.int32, 3),
    (3_000, 3, 10, 16, np.int32, 8), (10_000, 2, 7, 16, np.int32, 1 << 20),
    (9_000, 3, 16, 8, np.float32, 0), (6_000, 5, 5, 16, np.float32, 0), (4_000, 8, 33, 4, np.int32, 50),
])
def test_knn_graph(pg, dev, n, d, k, leaf, dtype, span):
    say(f"knn graph n={n} d={d} k={k} leaf={leaf} {dtype.__name__}")
    rng = np.random.default_rng(n + d * 7 + k)
    if dtype == np.int32:
        pts = rng.integers(0, span, (n, d)).astype(np.int32)
    else:
        pts = rng.standard_normal((n, d)).astype(np.float32)
    t = pg.kdtree_build(to_dev(pts, dev), leaf=leaf)
    gi, gd = host(*t.knn_graph(k))
    oi, od = oracle.knn_graph_brute(pts, k, nthreads=8)
    assert not np.any(gi == np.arange(n)[:, None])
    if dtype == np.int32:
        assert_int_equal(gi, gd, oi, od)
    else:
        assert_float_close(gi, gd, oi, od, pts, pts)


def test_knn_graph_full_size_sampled(pg, dev):
    # the headline shape (10M 3-D int uniform, leaf 16), k = 10, no self edges
    pts = datagen.uniform_int(10_000_000, 3, seed=2)
    say("knn graph 10M 3-D")
    t = pg.kdtree_build(to_dev(pts, dev), leaf=16)
    gi, gd = host(*t.knn_graph(10))
    assert (gi >= 0).all() and (np.diff(gd, axis=1) >= 0).all()
    assert not np.any(gi == np.arange(len(pts))[:, None])
    rows = np.random.default_rng(12).choice(len(pts), 300, replace=False)
    oi, od = graph_oracle_rows(pts, rows, 10)
    assert_int_equal(gi[rows], gd[rows], oi, od)


@pytest.mark.parametrize("case", range(0, 36, 3))
def test_wave_walk_small_random(pg, dev, case, monkeypatch):
    # the wave-per-block walk (selected per launch by PG_KNN_WAVE) must
    # return the lists of the per-lane walk: all-points, separate queries
    # and queries equal to the points, over the mixed small cases
    monkeypatch.setenv("PG_KNN_WAVE", "both")
    for c in (case, case + 1, case + 2):
        test_small_random(pg, dev, c)


def test_wave_walk_ties_redo_graph(pg, dev, monkeypatch):
    monkeypatch.setenv("PG_KNN_WAVE", "both")
    test_ties_identical_grid_planes(pg, dev)
    test_wide_distances_exact_redo(pg, dev)
    say("wave walk: knn graph")
    pts = np.random.default_rng(4).integers(0, 8, (3_000, 3)).astype(np.int32)
    t = pg.kdtree_build(to_dev(pts, dev), leaf=16)
    gi, gd = host(*t.knn_graph(10))
    oi, od = oracle.knn_graph_brute(pts, 10, nthreads=8)
    assert_int_equal(gi, gd, oi, od)
