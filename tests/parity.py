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


def assert_float_close(g_idx, g_dist, o_ids, o_dist, points, queries, chunk=1 << 19):
    """float32 rows against the FP64 oracle's rows (every row):
    (i)   rank-wise |g_r - o_r| <= 1e-6 o_r (o_r = 0 => g_r = 0);
    (ii)  ids in only one of the two sets have an FP64 distance within
          [o_k (1 - 1e-6), o_k (1 + 1e-6)] (near-ties of the k-th distance);
    (iii) ids distinct, padding where the oracle pads;
    (iv)  every returned id's FP64 distance, recomputed from the points,
          matches the distance returned beside it within 1e-6;
    (v)   rows ascend by (distance, id): equal float32 distances in id order.
    Returns the number of rows whose id sets differ from the oracle's."""
    g_idx = np.asarray(g_idx).astype(np.int64)
    g_dist = np.asarray(g_dist).astype(np.float64)
    o_ids = np.asarray(o_ids)
    o_dist = np.asarray(o_dist)
    m, k = g_idx.shape
    if m == 0:
        return 0
    assert np.array_equal(g_idx < 0, o_ids < 0), "padding differs"
    P = np.asarray(points, dtype=np.float64)
    Q = np.asarray(queries, dtype=np.float64)
    ndiff = 0
    for a in range(0, m, chunk):
        b = min(m, a + chunk)
        gi, gd, oi, od = g_idx[a:b], g_dist[a:b], o_ids[a:b], o_dist[a:b]
        real = oi >= 0
        # (i) rank-wise distances
        o = np.where(real, od, 0.0)
        g = np.where(real, gd, 0.0)
        zero = o == 0
        assert np.all(g[zero] == 0), "zero distance not reproduced"
        rel = np.abs(g - o) / np.where(zero, 1.0, o)
        assert rel.max() <= REL, f"max rank-wise relative error {rel.max():.3e}"
        # (iv) returned distance against the FP64 distance of the returned id
        diff = Q[a:b, None, :] - P[np.where(real, gi, 0)]
        d64 = np.where(real, np.sum(diff * diff, axis=2), 0.0)
        z64 = d64 == 0
        rel = np.abs(g - d64) / np.where(z64, 1.0, d64)
        assert np.all(g[z64 & real] == 0) and rel.max() <= REL, \
            f"a returned distance differs from its id's distance (max rel {rel.max():.3e})"
        # (iii) distinct ids; (v) ascending (distance, id)
        srt = np.sort(np.where(real, gi, -1 - np.arange(k)), axis=1)
        assert np.all(np.diff(srt, axis=1) != 0), "duplicate ids"
        both = real[:, 1:] & real[:, :-1]
        up = (gd[:, 1:] > gd[:, :-1]) | ((gd[:, 1:] == gd[:, :-1]) & (gi[:, 1:] > gi[:, :-1]))
        assert np.all(up | ~both), "rows not ascending by (distance, id)"
        # (ii) differing ids only among near-ties of the k-th distance
        diff_rows = np.nonzero((np.sort(gi, axis=1) != np.sort(oi, axis=1)).any(axis=1))[0]
        ndiff += len(diff_rows)
        for r in diff_rows:
            gs = set(gi[r][gi[r] >= 0].tolist())
            os_ = set(oi[r][oi[r] >= 0].tolist())
            ok = od[r][real[r]].max()
            for j in gs ^ os_:
                dj = float(np.sum((Q[a + r] - P[j]) ** 2))
                assert ok * (1 - REL) <= dj <= ok * (1 + REL), (a + r, j, dj, ok)
    return ndiff
