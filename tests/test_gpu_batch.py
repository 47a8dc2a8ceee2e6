"""GPU parity of the batched-clouds form (one persistent launch) and of the
differentiable k-NN backward, against the CPU oracle (FP64) and against the
per-cloud static path."""
import numpy as np
import pytest

import oracle
from oracle.grad import fd_self_incremental, grad_closed_form
from paper_2207_01834_amd import datagen
from parity import assert_float_close, say

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


def small_clouds(seed, C=150, hi=3000):
    g = np.random.default_rng(seed)
    sizes = np.floor(np.exp(g.uniform(0, np.log(hi), size=C))).astype(np.int64)
    sizes[:6] = [0, 1, 2, 15, 16, 17]  # empty, single, fewer than k, around the leaf size
    pts, offs = datagen.sphere_clouds(sizes, seed)
    return pts, offs


def per_cloud_static(pg, dev, pts, offs, k):
    """The plain per-cloud method: one static build + all-points k-NN each."""
    N = len(pts)
    gi = np.full((N, k), -1, np.int64)
    gd = np.full((N, k), np.inf, np.float64)
    for c in range(len(offs) - 1):
        a, b = int(offs[c]), int(offs[c + 1])
        if b == a:
            continue
        t = pg.kdtree_build(to_dev(pts[a:b], dev), leaf=16)
        i, d = host(*t.knn_all(k))
        gi[a:b] = np.where(i >= 0, i.astype(np.int64) + a, -1)
        gd[a:b] = d
    return gi, gd


def oracle_per_cloud(pts, offs, k, rows=None):
    """FP64 definition within each cloud; ids are global rows."""
    N = len(pts)
    cl = np.searchsorted(offs, np.arange(N), side="right") - 1
    rows = np.arange(N) if rows is None else rows
    oi = np.empty((len(rows), k), np.int64)
    od = np.empty((len(rows), k), np.float64)
    for c in np.unique(cl[rows]):
        a, b = int(offs[c]), int(offs[c + 1])
        sel = np.nonzero(cl[rows] == c)[0]
        ids, dist = oracle.knn_brute(pts[a:b], pts[rows[sel]], k, nthreads=8)
        oi[sel] = np.where(ids >= 0, ids + a, -1)
        od[sel] = dist
    return oi, od


def test_batched_matches_oracle_and_static(pg, dev):
    pts, offs = small_clouds(11)
    k = 16
    B = pg.BatchKnn(offs, 3, device=dev)
    gi, gd = host(*B.knn_self(to_dev(pts, dev), k))
    assert not B.timed_out()
    oi, od = oracle_per_cloud(pts, offs, k)
    assert_float_close(gi, gd, oi, od, pts, pts)
    # bitwise identical to the per-cloud static method (same fp32 arithmetic)
    si, sd = per_cloud_static(pg, dev, pts, offs, k)
    assert np.array_equal(gi.astype(np.int64), si)
    assert np.array_equal(gd.astype(np.float64), sd)


def test_batched_tuning_invariance(pg, dev):
    pts, offs = small_clouds(12, C=60, hi=9000)
    ref = None
    for leaf in (8, 16, 32):
        for bpc in (1, 2, 4):
            for lq, kl in ((1, pg.KLIST_VGPR), (4, pg.KLIST_LDS), (3, pg.KLIST_VGPR), (1, pg.KLIST_LDS)):
                say(f"tune leaf={leaf} bpc={bpc} lane_queries={lq} klist={kl}")
                B = pg.BatchKnn(offs, 3, leaf=leaf, blocks_per_cu=bpc, lane_queries=lq, klist=kl,
                                device=dev)
                out = host(*B.knn_self(to_dev(pts, dev), 10))
                if ref is None:
                    ref = out
                assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])
    # the LDS list with a guarded (non-exact) capacity, against the register list
    for k in (7, 33):
        a = host(*pg.BatchKnn(offs, 3, klist=pg.KLIST_VGPR, device=dev).knn_self(to_dev(pts, dev), k))
        b = host(*pg.BatchKnn(offs, 3, klist=pg.KLIST_LDS, lane_queries=2, device=dev).knn_self(to_dev(pts, dev), k))
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    t = pg.batch_autotune(to_dev(pts, dev), offs, 10)
    assert t["leaf"] in (8, 16, 32) and t["blocks_per_cu"] in (2, 4)
    assert t["lane_queries"] in (1, 4) and t["klist"] in (pg.KLIST_VGPR, pg.KLIST_LDS)


def test_batched_other_dims_and_k(pg, dev):
    g = np.random.default_rng(13)
    for d, k in ((2, 1), (5, 7), (8, 33)):
        sizes = g.integers(0, 2500, size=40)
        offs = np.zeros(41, np.int64)
        offs[1:] = np.cumsum(sizes)
        pts = (g.standard_normal((int(offs[-1]), d))).astype(np.float32)
        B = pg.BatchKnn(offs, d, device=dev)
        gi, gd = host(*B.knn_self(to_dev(pts, dev), k))
        oi, od = oracle_per_cloud(pts, offs, k)
        assert_float_close(gi, gd, oi, od, pts, pts)


def test_batched_graph_capture_replays(pg, dev):
    import torch
    pts, offs = small_clouds(14, C=80)
    k = 8
    x = to_dev(pts, dev)
    B = pg.BatchKnn(offs, 3, device=dev)
    eager = host(*B.knn_self(x, k))
    idx = torch.empty((len(pts), k), dtype=torch.int32, device=dev)
    d2 = torch.empty((len(pts), k), dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.knn_self(x, k, out=(idx, d2))  # warm on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.knn_self(x, k, out=(idx, d2))
    for rep in range(3):
        idx.fill_(-7)
        d2.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = host(idx, d2)
        assert np.array_equal(got[0], eager[0]) and np.array_equal(got[1], eager[1]), rep
        _ = (x * 2).sum().item()  # eager work between replays


def test_cfg4_full_size(pg, dev):
    """4,096 clouds, sizes log-uniform in [256, 65536], k = 16, one launch:
    every row of 66 whole clouds (the largest, the smallest and 64 drawn at
    random) against the oracle's kd-tree search within the cloud."""
    sizes = datagen.cloud_sizes(4096, seed=4)
    pts, offs = datagen.sphere_clouds(sizes, seed=44)
    say(f"cfg4: {len(pts)} points")
    x = to_dev(pts, dev)
    B = pg.BatchKnn(offs, 3, device=dev)
    gi, gd = host(*B.knn_self(x, 16))
    assert not B.timed_out()
    assert (gi[:, 0] >= 0).all()
    pick = np.random.default_rng(0).choice(len(sizes), 64, replace=False)
    pick = np.unique(np.concatenate([pick, [np.argmax(sizes), np.argmin(sizes)]]))
    for c in pick:
        a, b = int(offs[c]), int(offs[c + 1])
        cloud = pts[a:b]
        oi, od, _ = oracle.KdTree(cloud, leaf=16).knn(cloud, 16, nthreads=16)
        assert_float_close(gi[a:b] - a, gd[a:b], oi, od, cloud, cloud)


def test_backward_fd_and_closed_form(pg, dev):
    """Autograd of sum g * kNN d2 on 64 clouds of 256 points (k = 16) against
    FP64 central differences (away from ties) on all 64 clouds and the FP64
    closed form with the GPU's neighbour sets."""
    import torch

    from paper_2207_01834_amd.diff import knn_sqdist
    sizes = np.full(64, 256, dtype=np.int64)
    pts, offs = datagen.sphere_clouds(sizes, seed=404)
    k = 16
    G = np.random.default_rng(1).standard_normal((len(pts), k)).astype(np.float32)
    x = to_dev(pts, dev).requires_grad_(True)
    d2, idx = knn_sqdist(x, k, offsets=offs)
    (d2 * to_dev(G, dev)).sum().backward()
    grad = host(x.grad)[0].astype(np.float64)
    idx_h = host(idx)[0].astype(np.int64)
    # closed form (FP64) with the GPU's neighbour sets, both roles
    gq, gx = grad_closed_form(pts, pts, idx_h, G)
    cf = gq + gx
    scale = np.abs(cf).max()
    assert np.all(np.abs(grad - cf) <= 1e-4 * np.abs(cf) + 1e-4 * scale)
    # FP64 central differences on every cloud
    for c in range(len(sizes)):
        a, b = int(offs[c]), int(offs[c + 1])
        fd, stable = fd_self_incremental(pts[a:b].astype(np.float64), k, G[a:b].astype(np.float64),
                                         h=1e-6)
        sub = grad[a:b]
        assert stable.mean() > 0.8
        err = np.abs(sub - fd)[stable]
        assert np.all(err <= 1e-4 * np.abs(fd)[stable] + 1e-4 * np.abs(fd).max()), err.max()
    # deterministic: a second backward gives identical bits
    x2 = to_dev(pts, dev).requires_grad_(True)
    d2b, _ = knn_sqdist(x2, k, offsets=offs)
    (d2b * to_dev(G, dev)).sum().backward()
    assert np.array_equal(host(x2.grad)[0], host(x.grad)[0])


@pytest.mark.parametrize("d,k", [(3, 16), (3, 7), (5, 10)])
def test_batched_backward_leaf_order(pg, dev, d, k):
    """pg_batch_backward (leaf-order windows, int64 fixed point) against the
    FP64 closed form with the GPU's neighbour sets, on uneven clouds with an
    empty cloud, clouds smaller than k and a cloud of identical points (its
    first k rows are every point's neighbours: far outside any window); and
    against the generic backward; deterministic over two calls."""
    import torch
    g = np.random.default_rng(40 + d + k)
    sizes = np.floor(np.exp(g.uniform(0, np.log(9000), size=40))).astype(np.int64)
    sizes[:4] = [0, 3, 2500, 6000]
    if d == 3:
        pts, offs = datagen.sphere_clouds(sizes, 40 + k)
    else:
        offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        pts = g.standard_normal((int(offs[-1]), d)).astype(np.float32)
    a, b = int(offs[2]), int(offs[3])
    pts[a:b] = pts[a]  # identical points
    G = g.standard_normal((len(pts), k)).astype(np.float32)
    B = pg.BatchKnn(offs, d, device=dev)
    x = to_dev(pts, dev)
    idx, d2 = B.knn_self(x, k)
    gb = B.backward(x, idx, d2, to_dev(G, dev))
    gb2 = B.backward(x, idx, d2, to_dev(G, dev))
    grad = host(gb)[0].astype(np.float64)
    assert np.array_equal(host(gb2)[0], host(gb)[0])
    idx_h = host(idx)[0].astype(np.int64)
    gq, gx = grad_closed_form(pts, pts, idx_h, G)
    cf = gq + gx
    scale = np.abs(cf).max()
    assert np.all(np.abs(grad - cf) <= 1e-5 * np.abs(cf) + 1e-5 * scale)
    gen, _ = pg.knn_backward(x, x, idx, to_dev(G, dev), self_mode=True)
    gen = host(gen)[0].astype(np.float64)
    assert np.all(np.abs(grad - gen) <= 1e-5 * np.abs(cf) + 1e-5 * scale)


def test_backward_query_form(pg, dev):
    import torch

    from paper_2207_01834_amd.diff import knn_sqdist
    g = np.random.default_rng(2)
    X = g.random((3000, 3)).astype(np.float32)
    Q = g.random((500, 3)).astype(np.float32)
    k = 6
    x = to_dev(X, dev).requires_grad_(True)
    q = to_dev(Q, dev).requires_grad_(True)
    d2, idx = knn_sqdist(x, k, queries=q)
    W = g.standard_normal((500, k)).astype(np.float32)
    (d2 * to_dev(W, dev)).sum().backward()
    gq_ref, gx_ref = grad_closed_form(Q, X, host(idx)[0].astype(np.int64), W)
    for got, ref in ((host(q.grad)[0], gq_ref), (host(x.grad)[0], gx_ref)):
        scale = np.abs(ref).max()
        assert np.all(np.abs(got - ref) <= 1e-4 * np.abs(ref) + 1e-4 * scale)


@pytest.mark.parametrize("self_mode", [False, True])
def test_backward_float_atomics(pg, dev, self_mode):
    # the float-atomic form against the FP64 closed form (same bar as the
    # deterministic one) and against the deterministic kernel, with padding
    import torch
    g = np.random.default_rng(5 + self_mode)
    X = g.random((4000, 3)).astype(np.float32)
    Q = X if self_mode else g.random((700, 3)).astype(np.float32)
    k = 8
    m = len(Q)
    idx = g.integers(0, len(X), (m, k)).astype(np.int32)
    idx[::7, -1] = -1  # padding slots are skipped
    W = g.standard_normal((m, k)).astype(np.float32)
    xd = to_dev(X, dev)
    qd = xd if self_mode else to_dev(Q, dev)  # one tensor in both roles
    args = (qd, xd, to_dev(idx, dev), to_dev(W, dev))
    gq_f, gp_f = pg.knn_backward(*args, self_mode=self_mode, deterministic=False)
    gq_d, gp_d = pg.knn_backward(*args, self_mode=self_mode)
    gq_f, gp_f, gq_d, gp_d = host(gq_f, gp_f, gq_d, gp_d)
    gq_ref, gx_ref = grad_closed_form(Q, X, idx, W)
    if self_mode:
        refs = [(gq_f, gq_ref + gx_ref), (gq_d, gq_ref + gx_ref)]
    else:
        refs = [(gq_f, gq_ref), (gp_f, gx_ref), (gq_d, gq_ref), (gp_d, gx_ref)]
    for got, ref in refs:
        scale = np.abs(ref).max()
        assert np.all(np.abs(got - ref) <= 1e-4 * np.abs(ref) + 1e-4 * scale)
    if not self_mode:
        assert np.array_equal(gq_f, gq_d)  # the per-query sums are the same kernel


# --- separate query sets per cloud (pg_batch_knn) ---------------------------

def query_sets(seed, offs, d=3):
    """Queries per cloud: uneven counts, clouds without queries, query-only
    clouds (no points), queries near the cloud's points and far from them."""
    g = np.random.default_rng(seed)
    C = len(offs) - 1
    counts = np.floor(np.exp(g.uniform(0, np.log(2000), size=C))).astype(np.int64)
    counts[6:9] = 0          # clouds with points but no queries
    counts[0] = 37           # the empty cloud is queried (padding rows)
    qo = np.zeros(C + 1, np.int64)
    qo[1:] = np.cumsum(counts)
    q = (g.standard_normal((int(qo[-1]), d)) * 1.2).astype(np.float32)
    return q, qo


def oracle_query_sets(pts, offs, q, qo, k):
    oi = np.full((len(q), k), -1, np.int64)
    od = np.full((len(q), k), np.inf, np.float64)
    for c in range(len(offs) - 1):
        a, b = int(offs[c]), int(offs[c + 1])
        qa, qb = int(qo[c]), int(qo[c + 1])
        if qb == qa or b == a:
            continue
        ids, dist = oracle.knn_brute(pts[a:b], q[qa:qb], k, nthreads=8)
        oi[qa:qb] = np.where(ids >= 0, ids + a, -1)
        od[qa:qb] = dist
    return oi, od


@pytest.mark.parametrize("d,k", [(3, 10), (3, 16), (2, 1), (5, 7), (8, 33)])
def test_batched_query_sets(pg, dev, d, k):
    say(f"query sets d={d} k={k}")
    if d == 3:
        pts, offs = small_clouds(21 + k, C=120)
    else:
        g = np.random.default_rng(22 + d)
        sizes = g.integers(0, 2500, size=50)
        sizes[0] = 0
        offs = np.zeros(51, np.int64)
        offs[1:] = np.cumsum(sizes)
        pts = g.standard_normal((int(offs[-1]), d)).astype(np.float32)
    q, qo = query_sets(30 + d + k, offs, d)
    B = pg.BatchKnn(offs, d, device=dev)
    gi, gd = host(*B.knn(to_dev(pts, dev), to_dev(q, dev), qo, k))
    assert not B.timed_out()
    oi, od = oracle_query_sets(pts, offs, q, qo, k)
    assert_float_close(gi, gd, oi, od, pts, q)
    # the self form on the same handle is unchanged, and the query form again
    si, sd = host(*B.knn_self(to_dev(pts, dev), k))
    oi2, od2 = oracle_per_cloud(pts, offs, k)
    assert_float_close(si, sd, oi2, od2, pts, pts)
    gi2, gd2 = host(*B.knn(to_dev(pts, dev), to_dev(q, dev), qo, k))
    assert np.array_equal(gi2, gi) and np.array_equal(gd2, gd)


def test_batched_query_sets_graph_replays_and_new_layout(pg, dev):
    import torch
    pts, offs = small_clouds(41, C=90)
    q, qo = query_sets(42, offs)
    k = 8
    x, qd = to_dev(pts, dev), to_dev(q, dev)
    B = pg.BatchKnn(offs, 3, device=dev)
    eager = host(*B.knn(x, qd, qo, k))  # uploads the query layout
    idx = torch.empty((len(q), k), dtype=torch.int32, device=dev)
    d2 = torch.empty((len(q), k), dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.knn(x, qd, qo, k, out=(idx, d2))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.knn(x, qd, qo, k, out=(idx, d2))
    for rep in range(3):
        idx.fill_(-7)
        d2.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = host(idx, d2)
        assert np.array_equal(got[0], eager[0]) and np.array_equal(got[1], eager[1]), rep
        _ = (x * 2).sum().item()
    # a different layout of the same queries (uploaded again)
    qo2 = qo.copy()
    qo2[1:-1] = np.minimum(qo[1:-1] + 5, qo[-1])
    qo2 = np.maximum.accumulate(qo2)
    gi, gd = host(*B.knn(x, qd, qo2, k))
    oi, od = oracle_query_sets(pts, offs, q, qo2, k)
    assert_float_close(gi, gd, oi, od, pts, q)


def test_batched_query_sets_gradient(pg, dev):
    """knn_sqdist with per-cloud query sets: gradients to queries and points
    against the FP64 closed form with the GPU's neighbour sets."""
    import torch

    from paper_2207_01834_amd.diff import knn_sqdist
    pts, offs = small_clouds(51, C=40, hi=1500)
    q, qo = query_sets(52, offs)
    k = 6
    x = to_dev(pts, dev).requires_grad_(True)
    qq = to_dev(q, dev).requires_grad_(True)
    d2, idx = knn_sqdist(x, k, offsets=offs, queries=qq, q_offsets=qo)
    W = np.random.default_rng(53).standard_normal((len(q), k)).astype(np.float32)
    real = host(idx)[0] >= 0
    # padding slots (query-only clouds) hold +inf: left out of the loss
    live = torch.where(to_dev(real, dev), d2, torch.zeros_like(d2))
    (live * to_dev(W * real, dev)).sum().backward()
    gq_ref, gx_ref = grad_closed_form(q, pts, host(idx)[0].astype(np.int64), W * real)
    for got, ref in ((host(qq.grad)[0], gq_ref), (host(x.grad)[0], gx_ref)):
        scale = np.abs(ref).max()
        assert np.all(np.abs(got - ref) <= 1e-4 * np.abs(ref) + 1e-4 * scale)


def test_batched_backward_mixed_scales_and_nonfinite(pg, dev):
    """Clouds of very different sizes in one batch (unit sphere, and scaled by
    1e3 and 1e-3): each cloud's gradients to a purely relative bar away from
    zero (the fixed-point scale is per cloud); a cloud whose gradient input
    holds a NaN gets NaN gradients and raises the status bit, the others are
    unaffected."""
    sizes = np.array([3000, 2500, 2000, 1500], dtype=np.int64)
    pts, offs = datagen.sphere_clouds(sizes, 61)
    pts = pts.astype(np.float64)
    pts[offs[1]:offs[2]] *= 1e3
    pts[offs[2]:offs[3]] *= 1e-3
    pts = pts.astype(np.float32)
    k = 10
    G = np.random.default_rng(62).standard_normal((len(pts), k)).astype(np.float32)
    B = pg.BatchKnn(offs, 3, device=dev)
    x = to_dev(pts, dev)
    idx, d2 = B.knn_self(x, k)
    grad = host(B.backward(x, idx, d2, to_dev(G, dev)))[0].astype(np.float64)
    assert not B.backward_nonfinite()
    idx_h = host(idx)[0].astype(np.int64)
    gq, gx = grad_closed_form(pts, pts, idx_h, G)
    cf = gq + gx
    for c in range(len(sizes)):
        a, b = int(offs[c]), int(offs[c + 1])
        ref, got = cf[a:b], grad[a:b]
        big = np.abs(ref) >= 1e-3 * np.abs(ref).max()
        rel = np.abs(got - ref)[big] / np.abs(ref)[big]
        assert rel.max() <= 1e-4, (c, rel.max())
    Gn = G.copy()
    Gn[offs[3] + 5, 2] = np.nan
    grad = host(B.backward(x, idx, d2, to_dev(Gn, dev)))[0]
    assert B.backward_nonfinite()
    assert np.isnan(grad[offs[3]:offs[4]]).all()
    assert np.isfinite(grad[:offs[3]]).all()


_TUNE_CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
from paper_2207_01834_amd import _binding as pg, datagen
sizes = np.array([300, 0, 1500, 40, 900], dtype=np.int64)
pts, offs = datagen.sphere_clouds(sizes, 5)
x = torch.from_numpy(pts).to("cuda:0")
print(json.dumps(pg.batch_autotune(x, offs, 8)))
"""


def test_autotune_cache_file(pg, dev, tmp_path):
    # PG_TUNE_CACHE keeps the tuner's choice across processes: the first
    # process times and appends a line; a second one returns the file's
    # choice (here edited to another valid setting) without timing
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, PG_TUNE_CACHE=str(cache))

    def child():
        say("autotune child process")
        r = subprocess.run([sys.executable, "-c", _TUNE_CHILD, root], env=env, capture_output=True,
                           text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    first = child()
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    f = lines[0].split()
    assert len(f) == 9 and [int(v) for v in f[5:]] == [first["leaf"], first["blocks_per_cu"],
                                                        first["lane_queries"], first["klist"]]
    other = [8 if first["leaf"] != 8 else 32, 2, 4, pg.KLIST_LDS]
    cache.write_text("not a line\n" + " ".join(f[:5] + [str(v) for v in other]) + "\n")
    second = child()
    assert [second["leaf"], second["blocks_per_cu"], second["lane_queries"], second["klist"]] == other
    assert len(cache.read_text().splitlines()) == 2  # found: nothing appended
