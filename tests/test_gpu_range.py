"""GPU parity of the orthogonal range search (pg_range_count,
pg_range_report and pg_range_search through the C ABI) against the CPU oracle's definition:
counts and reported rows bit-exact (no arithmetic, only comparisons, so
float32 is exact too), rows in the tree's leaf order, edge cases, the
overflow guard and full-size sampled boxes."""
import numpy as np
import pytest

import oracle
from paper_2207_01834_amd import datagen
from parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pg(dev):
    import paper_2207_01834_amd._binding as b
    b.lib()
    return b


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def check_case(pg, dev, pts, boxes, leaf):
    say(f"range case n={len(pts)} d={pts.shape[1]} m={len(boxes)} leaf={leaf} dtype={pts.dtype}")
    import torch
    t = pg.kdtree_build(to_dev(pts, dev), leaf=leaf)
    B = to_dev(boxes, dev)
    counts, off, total = t.range_count(B, offsets=True)
    plain = t.range_count(B)
    o_rows, rows = t.range_search(B)
    torch.cuda.synchronize()
    counts, off, plain, o_rows, rows = [x.cpu().numpy() for x in (counts, off, plain, o_rows, rows)]
    oc, oo, oi = oracle.range_brute(pts, boxes)
    assert np.array_equal(counts.astype(np.int64), oc), f"counts differ at {np.nonzero(counts != oc)[0][:5]}"
    assert np.array_equal(plain, counts)
    assert np.array_equal(off, oo) and total == int(oo[-1])
    assert np.array_equal(o_rows, oo)
    assert rows.shape[0] == total
    # rows: the same set per box, in the tree's leaf order
    _, perm = t.export()
    pos = np.empty(len(pts), dtype=np.int64)
    pos[perm.astype(np.int64)] = np.arange(len(pts))
    for i in range(len(boxes)):
        g = rows[oo[i]:oo[i + 1]].astype(np.int64)
        assert np.array_equal(np.sort(g), oi[oo[i]:oo[i + 1]]), f"box {i} rows differ"
        assert np.all(np.diff(pos[g]) > 0), f"box {i} rows not in leaf order"
    return t


@pytest.mark.parametrize("d,leaf,dtype,n", [
    (2, 16, np.int32, 20_000), (3, 16, np.int32, 12_345), (2, 8, np.float32, 9_999),
    (5, 16, np.float32, 7_000), (1, 4, np.int32, 3_000), (8, 3, np.int32, 2_500),
    (4, 64, np.float32, 5_000), (7, 1, np.int32, 1_000),
])
def test_random_boxes(pg, dev, d, leaf, dtype, n):
    rng = np.random.default_rng(1000 + d * 17 + leaf)
    if dtype == np.int32:
        pts = datagen.uniform_int(n, d, seed=d + leaf, bits=12)
        half = 1 << 11 if d > 3 else 700
    else:
        pts = rng.standard_normal((n, d)).astype(np.float32)
        half = 1.2 if d > 3 else 0.5
    boxes = datagen.range_boxes(pts, half, seed=7 + d, m=5_000)
    boxes[0] = [pts.min(0), pts.max(0)]
    boxes[1] = [pts.max(0), pts.min(0)]
    boxes[2] = [pts[5], pts[5]]
    check_case(pg, dev, pts, boxes, leaf)


def test_all_points_squares_2d(pg, dev):
    # the all-points workload shape at a size the oracle finishes quickly
    pts = datagen.uniform_int(30_000, 2, seed=2, bits=14)
    boxes = datagen.range_boxes(pts, 40)
    check_case(pg, dev, pts, boxes, 16)


def test_duplicates_and_small_trees(pg, dev):
    rng = np.random.default_rng(3)
    pts = rng.integers(0, 4, (3_000, 3)).astype(np.int32)
    boxes = datagen.range_boxes(pts, 2, seed=4, m=600)
    check_case(pg, dev, pts, boxes, 16)
    for n, leaf in [(1, 16), (2, 1), (5, 1), (17, 4), (64, 64), (65, 64)]:
        p = rng.integers(-50, 50, (n, 2)).astype(np.int32)
        b = datagen.range_boxes(p, 30, seed=n, m=50)
        check_case(pg, dev, p, b, leaf)


def test_float_signed_zero(pg, dev):
    pts = np.array([[0.0, 1.0], [-0.0, 1.0], [1.5, -0.0], [-1.5, 0.0]] * 10, dtype=np.float32)
    boxes = np.array([[[-0.0, -0.0], [0.0, 1.0]], [[0.0, 0.0], [1.5, 0.0]],
                      [[-1.5, -0.0], [-0.0, 0.0]]], dtype=np.float32)
    check_case(pg, dev, pts, boxes, 2)


def test_empty_tree_and_no_boxes(pg, dev):
    import torch
    t = pg.kdtree_build(to_dev(np.zeros((0, 2), dtype=np.int32), dev), leaf=16)
    b = to_dev(datagen.range_boxes(datagen.uniform_int(10, 2, seed=1), 5, seed=1, m=10), dev)
    counts, off, total = t.range_count(b, offsets=True)
    o, rows = t.range_search(b)
    torch.cuda.synchronize()
    assert counts.cpu().tolist() == [0] * 10 and total == 0 and rows.numel() == 0
    assert off.cpu().tolist() == [0] * 11
    t2 = pg.kdtree_build(to_dev(datagen.uniform_int(100, 2, seed=2), dev), leaf=16)
    c, off, total = t2.range_count(b[:0], offsets=True)
    assert c.numel() == 0 and total == 0 and off.cpu().tolist() == [0]


def test_bad_boxes_and_overflow_guard(pg, dev):
    import torch
    pts = datagen.uniform_int(5_000, 2, seed=9, bits=10)
    t = pg.kdtree_build(to_dev(pts, dev), leaf=16)
    bad = datagen.range_boxes(pts, 10, seed=2, m=8)
    bad[3, 1, 0] = 1 << 29
    with pytest.raises(pg.RangeError):
        t.range_count(to_dev(bad, dev))
    boxes = to_dev(datagen.range_boxes(pts, 60, seed=3, m=100), dev)
    counts, off, total = t.range_count(boxes, offsets=True)
    assert total > 10
    out = torch.full((total - 1,), -7, dtype=torch.int32, device=dev)
    with pytest.raises(pg.PargeoError):
        t.range_report(boxes, off, out)
    # every slot below the capacity was written
    full = torch.empty(total, dtype=torch.int32, device=dev)
    t.range_report(boxes, off, full)
    torch.cuda.synchronize()
    assert torch.equal(out, full[:total - 1])


def test_full_size_2d_sampled(pg, dev):
    """The all-points 2-D workload at full size (10M uniform points in
    [0, 2^20)^2, a square of half side 512 around every point): sampled boxes
    against the oracle, totals and containment of every reported row of the
    first million boxes."""
    import torch
    n = 10_000_000
    pts = datagen.uniform_int(n, 2, seed=2)
    say("full-size range: build")
    P = to_dev(pts, dev)
    t = pg.kdtree_build(P, leaf=16)
    boxes = datagen.range_boxes(pts, 512)
    B = to_dev(boxes, dev)
    say("full-size range: count + report")
    counts, off, total = t.range_count(B, offsets=True)
    _, rows = t.range_search(B)
    torch.cuda.synchronize()
    counts = counts.cpu().numpy().astype(np.int64)
    off = off.cpu().numpy()
    assert off[-1] == total == counts.sum()
    assert counts.min() >= 1  # every box holds its centre
    say(f"full-size range: total {total}, mean {total / n:.2f}")
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(n, 40, replace=False))
    oc, oo, oi = oracle.range_brute(pts, boxes[sample])
    assert np.array_equal(counts[sample], oc)
    r_host = rows.cpu().numpy()
    for s, i in enumerate(sample):
        g = np.sort(r_host[off[i]:off[i + 1]].astype(np.int64))
        assert np.array_equal(g, oi[oo[s]:oo[s + 1]])
    # containment of every row reported for the first 1M boxes
    lim = int(off[1_000_000])
    owner = np.repeat(np.arange(1_000_000), counts[:1_000_000])
    p = pts[r_host[:lim]]
    lo, hi = boxes[owner, 0], boxes[owner, 1]
    assert np.all((p >= lo) & (p <= hi))


def test_search_capacity_fallback(pg, dev):
    """pg_range_search: a capacity below the total writes counts and offsets
    and leaves the rows to the reporting pass (the binding's fallback); an
    exact capacity does both passes in one call."""
    import torch
    pts = datagen.uniform_int(8_000, 3, seed=21, bits=10)
    t = pg.kdtree_build(to_dev(pts, dev), leaf=8)
    boxes = datagen.range_boxes(pts, 90, seed=22, m=3_000)
    B = to_dev(boxes, dev)
    oc, oo, oi = oracle.range_brute(pts, boxes)
    total = int(oo[-1])
    for cap in (0, 5, total - 1, total, total + 100):
        off, rows = t.range_search(B, capacity=cap)
        torch.cuda.synchronize()
        off, rows = off.cpu().numpy(), rows.cpu().numpy()
        assert np.array_equal(off, oo) and rows.shape[0] == total
        for i in range(0, 3_000, 37):
            assert np.array_equal(np.sort(rows[off[i]:off[i + 1]].astype(np.int64)), oi[oo[i]:oo[i + 1]])
