"""Pins for the CPU oracle's orthogonal range query (the definition written
out, and the same query on the oracle's kd-tree), checked against lattice
closed forms, a sorted-array search (NumPy's searchsorted) for d = 1,
special cases and invariants."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2207_01834_amd import datagen


def lattice(G, s, d):
    axes = [np.arange(G) * s] * d
    return np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, d).astype(np.int32)


def lattice_ids(G, s, lo, hi):
    # rows of the lattice points inside [lo, hi]: per axis the multiples t*s
    # in range, then the row-major index of each combination
    per_axis = []
    for a, b in zip(lo, hi):
        t0 = max(0, -(-int(a) // s))
        t1 = min(G - 1, int(b) // s)
        per_axis.append(range(t0, t1 + 1))
    d = len(lo)
    out = []
    for t in itertools.product(*per_axis):
        out.append(sum(int(tc) * G ** (d - 1 - c) for c, tc in enumerate(t)))
    return sorted(out)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_lattice_counts_and_ids(d):
    G, s = 9, 5
    pts = lattice(G, s, d)
    rng = np.random.default_rng(10 + d)
    m = 60
    lo = rng.integers(-8, G * s + 3, (m, d))
    hi = lo + rng.integers(-3, 25, (m, d))
    # boxes whose faces sit exactly on lattice planes (closed on both sides)
    lo[:10] = (lo[:10] // s) * s
    hi[:10] = lo[:10] + s * rng.integers(0, 4, (10, d))
    boxes = np.stack([lo, hi], axis=1).astype(np.int32)
    counts, off, ids = oracle.range_brute(pts, boxes)
    for i in range(m):
        want = lattice_ids(G, s, lo[i], hi[i])
        assert counts[i] == len(want)
        assert ids[off[i]:off[i + 1]].tolist() == want


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_one_dimension_matches_sorted_search(dtype):
    rng = np.random.default_rng(7)
    x = rng.integers(-50, 50, 400)
    pts = x.astype(dtype).reshape(-1, 1)
    lo = rng.integers(-60, 60, 200)
    hi = lo + rng.integers(-5, 40, 200)
    boxes = np.stack([lo, hi], axis=1).astype(dtype).reshape(-1, 2, 1)
    counts, off, ids = oracle.range_brute(pts, boxes)
    srt = np.sort(x)
    want = np.maximum(np.searchsorted(srt, hi, "right") - np.searchsorted(srt, lo, "left"), 0)
    assert counts.tolist() == want.tolist()
    for i in range(200):
        got = ids[off[i]:off[i + 1]]
        assert np.all(np.diff(got) > 0)
        assert np.all((x[got] >= lo[i]) & (x[got] <= hi[i]))


def test_special_cases():
    pts = np.array([[0, 0], [1, 1], [1, 1], [2, -3], [5, 5]], dtype=np.int32)
    boxes = np.array([
        [[-9, -9], [9, 9]],      # everything
        [[3, 3], [2, 9]],        # lo > hi in x: empty
        [[1, 1], [1, 1]],        # a single location holding two points
        [[2, -3], [2, -3]],      # a single point, corners equal
        [[6, 6], [9, 9]],        # misses every point
    ], dtype=np.int32)
    counts, off, ids = oracle.range_brute(pts, boxes)
    assert counts.tolist() == [5, 0, 2, 1, 0]
    assert ids.tolist() == [0, 1, 2, 3, 4, 1, 2, 3]
    # ids and liveness
    alive = np.array([1, 0, 1, 1, 1], dtype=np.uint8)
    counts, off, ids = oracle.range_brute(pts, boxes, ids=np.arange(5) + 100, alive=alive)
    assert counts.tolist() == [4, 0, 1, 1, 0]
    assert ids.tolist() == [100, 102, 103, 104, 102, 103]


def test_float_signed_zero_and_edges():
    pts = np.array([[0.0], [-0.0], [1.5], [-1.5], [np.nextafter(np.float32(1.5), np.float32(2))]],
                   dtype=np.float32)
    boxes = np.array([[[-0.0], [-0.0]], [[0.0], [1.5]], [[-1.5], [-0.0]]], dtype=np.float32)
    counts, off, ids = oracle.range_brute(pts, boxes)
    assert counts.tolist() == [2, 3, 3]
    assert ids.tolist() == [0, 1, 0, 1, 2, 0, 1, 3]


def test_empty_inputs():
    pts = np.zeros((0, 3), dtype=np.int32)
    counts, off, ids = oracle.range_brute(pts, np.zeros((4, 2, 3), dtype=np.int32))
    assert counts.tolist() == [0] * 4 and ids.size == 0
    pts = np.ones((5, 3), dtype=np.int32)
    counts, off, ids = oracle.range_brute(pts, np.zeros((0, 2, 3), dtype=np.int32))
    assert counts.size == 0 and off.tolist() == [0]


def _boxes_around(rng, pts, m, half):
    c = pts[rng.integers(0, pts.shape[0], m)].astype(np.float64)
    w = rng.uniform(0, half, (m, pts.shape[1]))
    lo, hi = c - w, c + w
    return np.stack([lo, hi], axis=1).astype(pts.dtype)


@pytest.mark.parametrize("d,leaf,dtype", [(1, 4, np.int32), (2, 16, np.int32), (3, 1, np.int32),
                                          (2, 8, np.float32), (5, 16, np.float32),
                                          (8, 3, np.int32)])
def test_tree_range_equals_definition(d, leaf, dtype):
    rng = np.random.default_rng(100 + d * 10 + leaf)
    n = 3000
    if dtype == np.int32:
        pts = rng.integers(-1000, 1000, (n, d)).astype(np.int32)
        pts[::7] = pts[3]  # many duplicates
        half = 300
    else:
        pts = rng.standard_normal((n, d)).astype(np.float32)
        half = 0.8
    boxes = _boxes_around(rng, pts, 300, half)
    boxes[0, 0], boxes[0, 1] = pts.min(axis=0), pts.max(axis=0)
    boxes[1, 0], boxes[1, 1] = pts.max(axis=0), pts.min(axis=0)
    cb, ob, ib = oracle.range_brute(pts, boxes)
    T = oracle.KdTree(pts, leaf=leaf)
    ct, ot, it, counters = T.range(boxes)
    assert ct.tolist() == cb.tolist()
    assert ct[0] == n and ct[1] == (n if np.all(pts.min(0) == pts.max(0)) else 0)
    for i in range(boxes.shape[0]):
        assert sorted(it[ot[i]:ot[i + 1]].tolist()) == ib[ob[i]:ob[i + 1]].tolist()
    # the tree tests far fewer points than the n per box of the definition
    assert counters[1] < 0.5 * n * boxes.shape[0]


def test_tree_range_whole_box_tests_only_the_root():
    pts = datagen.uniform_int(5000, 2, seed=3)
    T = oracle.KdTree(pts, leaf=16)
    boxes = np.array([[pts.min(0), pts.max(0)]], dtype=np.int32)
    c, o, ids, counters = T.range(boxes)
    assert c[0] == 5000 and counters.tolist() == [1, 0]
    assert sorted(ids.tolist()) == list(range(5000))


def test_tree_range_live_subset():
    rng = np.random.default_rng(5)
    pts = rng.integers(0, 200, (2000, 2)).astype(np.int32)
    alive = (rng.random(2000) < 0.6).astype(np.uint8)
    ids = rng.permutation(2000).astype(np.int64) * 3
    boxes = _boxes_around(rng, pts, 100, 40)
    cb, ob, ib = oracle.range_brute(pts, boxes, ids=ids, alive=alive)
    ct, ot, it, _ = oracle.KdTree(pts, leaf=8).range(boxes, ids=ids, alive=alive)
    assert ct.tolist() == cb.tolist()
    for i in range(100):
        assert sorted(it[ot[i]:ot[i + 1]].tolist()) == sorted(ib[ob[i]:ob[i + 1]].tolist())
