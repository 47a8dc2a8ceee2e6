"""pg_knn_noalloc (k-NN for callers that cannot allocate) against pg_knn:
identical rows on the same trees and queries, two calls in a row (the
second smaller, so stale scratch contents would show), object- and
spatial-median trees, int32 (including queries whose packed keys clamp and
take the exact redo pass) and float32, and the size limit."""
import ctypes

import numpy as np
import pytest

from paper_2207_01834_amd import datagen
from parity import say

pytestmark = pytest.mark.gpu

MAX_Q = 1 << 22


@pytest.fixture(scope="module")
def pg(dev):
    import paper_2207_01834_amd._binding as b
    b.lib()
    return b


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def noalloc(pg, t, q, k):
    """One call of pg_knn_noalloc through the C ABI into fresh outputs."""
    import torch
    m = q.shape[0]
    idx = torch.full((m, k), -7, dtype=torch.int32, device=q.device)
    dist = torch.full((m, k), -7, dtype=torch.int64 if q.dtype == torch.int32 else torch.float32,
                      device=q.device)
    st = pg.lib().pg_knn_noalloc(t._h, ctypes.c_void_p(q.data_ptr()), m, k,
                                 ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                                 pg.stream_ptr(q.device))
    assert st == 0, pg.lib().pg_last_error()
    return idx, dist


def same(a, b):
    import torch
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())


@pytest.mark.parametrize("split", ["object", "spatial"])
@pytest.mark.parametrize("dtype", ["int", "float"])
def test_noalloc_matches_knn_twice(pg, dev, split, dtype):
    say(f"noalloc {split} {dtype}")
    pts = datagen.uniform_int(300_000, 3, seed=71)
    rng = np.random.default_rng(72)
    q1 = rng.integers(0, 1 << 20, (120_000, 3)).astype(np.int32)
    q2 = rng.integers(0, 1 << 20, (9_000, 3)).astype(np.int32)
    if dtype == "float":
        pts, q1, q2 = (a.astype(np.float32) / (1 << 20) for a in (pts, q1, q2))
    t = pg.kdtree_build(to_dev(pts, dev), leaf=16, split=split)
    for q, k in ((q1, 10), (q2, 7)):  # the second call is smaller
        qd = to_dev(q, dev)
        same(noalloc(pg, t, qd, k), t.knn(qd, k))


def test_noalloc_redo_and_small(pg, dev):
    # coordinates near +-2^29: squared distances need more bits than the
    # packed keys leave, so every query takes the exact redo pass
    rng = np.random.default_rng(73)
    pts = rng.integers(-(1 << 29), 1 << 29, (50_000, 3)).astype(np.int32)
    t = pg.kdtree_build(to_dev(pts, dev), leaf=8)
    for m, k in ((20_000, 16), (5_000, 3), (100, 33)):
        q = to_dev(rng.integers(-(1 << 29), 1 << 29, (m, 3)).astype(np.int32), dev)
        same(noalloc(pg, t, q, k), t.knn(q, k))


def test_noalloc_limits(pg, dev):
    import torch
    t = pg.kdtree_build(to_dev(datagen.uniform_int(1_000, 2, seed=74), dev), leaf=16)
    q = to_dev(datagen.uniform_int(8, 2, seed=75), dev)
    idx = torch.empty((8, 4), dtype=torch.int32, device=dev)
    dist = torch.empty((8, 4), dtype=torch.int64, device=dev)
    st = pg.lib().pg_knn_noalloc(t._h, ctypes.c_void_p(q.data_ptr()), MAX_Q + 1, 4,
                                 ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                                 pg.stream_ptr(q.device))
    assert st == 1 and b"2^22" in pg.lib().pg_last_error()
    # the binding's form into caller tensors
    pg_i, pg_d = t.knn(q, 4)
    t.knn_noalloc(q, 4, (idx, dist))
    same((idx, dist), (pg_i, pg_d))
