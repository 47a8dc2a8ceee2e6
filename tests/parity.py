"""Comparison helpers for the GPU parity tests (element-wise against the CPU
oracle).  Bars:
  * int32 coordinates: byte-identical neighbour rows and int64 distances;
  * float32 coordinates against the FP64 oracle: per rank
    |g_r - o_r| <= 1e-6 o_r (o_r = 0 => g_r = 0); neighbour sets may differ
    only in ids whose FP64 distance lies within [o_k(1-1e-6), o_k(1+1e-6)];
    ids distinct; distances non-decreasing.
"""
import sys

import numpy as np

import oracle

REL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def leaf_keys(perm, n, L):
    sizes = np.diff(np.array([(j * n) >> L for j in range((1 << L) + 1)], dtype=np.int64))
    leaf_of = np.repeat(np.arange(1 << L, dtype=np.int64), sizes)
    return np.sort(leaf_of * max(n, 1) + perm.astype(np.int64))


def compare_tree(gpu_tree, points, leaf):
    """Split values and leaf membership identical to the oracle's tree."""
    t = oracle.KdTree(points, leaf=leaf)
    assert gpu_tree.levels == t.levels, (gpu_tree.levels, t.levels)
    sg, pg_ = gpu_tree.export()
    so, po = t.export()
    assert np.array_equal(sg.astype(np.float64), so), "split values differ"
    assert np.array_equal(leaf_keys(pg_, len(points), t.levels), leaf_keys(po, len(points), t.levels)), \
        "leaf membership differs"
    return t


def assert_int_equal(g_idx, g_dist, o_ids, o_dist):
    g_idx = np.asarray(g_idx).astype(np.int64)
    g_dist = np.asarray(g_dist)
    bad = np.nonzero((g_idx != o_ids).any(axis=1) | (g_dist != o_dist).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} rows differ, first {bad[:5]}: gpu {g_idx[bad[0]]} {g_dist[bad[0]]} oracle {o_ids[bad[0]]} {o_dist[bad[0]]}"


def assert_float_close(g_idx, g_dist, o_ids, o_dist, points, queries):
    g_idx = np.asarray(g_idx).astype(np.int64)
    g_dist = np.asarray(g_dist).astype(np.float64)
    m, k = g_idx.shape
    if m == 0:
        return 0
    # padding positions agree
    assert np.array_equal(g_idx < 0, o_ids < 0)
    real = o_ids >= 0
    # (iii) distances non-decreasing over the real entries
    steps = np.diff(np.where(real, g_dist, np.inf), axis=1)
    assert np.all((steps >= 0) | np.isnan(steps))
    # (i) rank-wise distances
    o = np.where(real, o_dist, 0.0)
    g = np.where(real, g_dist, 0.0)
    zero = o == 0
    assert np.all(g[zero] == 0), "zero distance not reproduced"
    rel = np.abs(g - o) / np.where(zero, 1.0, o)
    assert rel.max() <= REL, f"max rank-wise relative error {rel.max():.3e}"
    # (ii) differing ids only among near-ties of the k-th distance
    P = np.asarray(points, dtype=np.float64)
    Q = np.asarray(queries, dtype=np.float64)
    diff_rows = np.nonzero((np.sort(g_idx, axis=1) != np.sort(o_ids, axis=1)).any(axis=1))[0]
    for r in diff_rows:
        gs = set(g_idx[r][g_idx[r] >= 0].tolist())
        os_ = set(o_ids[r][o_ids[r] >= 0].tolist())
        assert len(gs) == int((g_idx[r] >= 0).sum()), "duplicate ids"
        ok = o_dist[r][real[r]].max()
        for j in gs ^ os_:
            dj = float(np.sum((Q[r] - P[j]) ** 2))
            assert ok * (1 - REL) <= dj <= ok * (1 + REL), (r, j, dj, ok)
    return len(diff_rows)
