"""GPU parity of the BDL-tree (Section 5, Algorithms 3 and 4) against the
oracle's BDL model: per-step state (F, buffer count, live points per tree),
erase counts, and k-NN over the live points (byte-identical for int32)."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.bdl_model import BDLModel
from paper_2207_01834_amd import datagen
from parity import assert_float_close, assert_int_equal, say

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "bdl_insert_example.json")


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


def same_state(G, M, tag=""):
    gF, gb, glive = G.stats(40)
    mF, mb, mlive = M.stats(40)
    assert (gF, gb) == (mF, mb), f"{tag}: F/buffer gpu {(gF, gb)} model {(mF, mb)}"
    assert glive == mlive, f"{tag}: live per tree gpu {glive} model {mlive}"
    assert G.size() == M.size()


def knn_check(pg, dev, G, M, q, k):
    gi, gd = host(*G.knn(to_dev(q, dev), k))
    pts, ids = M.live()
    oi, od = oracle.knn_brute(pts, q, k, ids=ids, nthreads=8)
    assert_int_equal(gi, gd, oi, od)


def test_paper_insert_example(pg, dev):
    import torch
    gold = json.load(open(GOLD))
    X = 8
    g = np.random.default_rng(0)
    G = pg.BDLTree(2, torch.int32, leaf=4, X=X, device=dev)
    M = BDLModel(2, X)
    size = lambda e: eval(e, {"X": X})
    P = g.integers(0, 50, size=(size(gold["start"]["points"]), 2)).astype(np.int32)
    assert G.insert(to_dev(P, dev)) == M.insert(P) == 0
    same_state(G, M, "start")
    assert G.stats()[:2] == (gold["start"]["F"], gold["start"]["buffer"])
    for st in gold["steps"]:
        P = g.integers(0, 50, size=(size(st["insert"]), 2)).astype(np.int32)
        assert G.insert(to_dev(P, dev)) == M.insert(P)
        same_state(G, M, st["insert"])
        assert G.stats()[:2] == (st["F"], st["buffer"])
        knn_check(pg, dev, G, M, g.integers(0, 50, size=(40, 2)).astype(np.int32), 5)


def _run_sequence(pg, dev, d, X, steps, coord_hi, dtype, seed, k=7, leaf=8, split="object"):
    import torch
    g = np.random.default_rng(seed)
    say(f"BDL sequence d={d} X={X} leaf={leaf} {np.dtype(dtype).name} split={split}")
    G = pg.BDLTree(d, torch.int32 if dtype == np.int32 else torch.float32, leaf=leaf, X=X, device=dev,
                   split=split)
    M = BDLModel(d, X, dtype=dtype)

    def draw(cnt):
        if dtype == np.int32:
            return g.integers(0, coord_hi, size=(cnt, d)).astype(np.int32)
        return (np.floor(g.random((cnt, d)) * coord_hi) / coord_hi).astype(np.float32)

    for step in range(steps):
        op = step % 3
        if op != 2:
            P = draw(int(g.integers(0, 6 * X)))
            say(f"step {step}: insert {len(P)}")
            assert G.insert(to_dev(P, dev)) == M.insert(P)
        else:
            pts, _ = M.live()
            cnt = int(g.integers(0, max(1, len(pts) // 2)))
            E = pts[np.sort(g.choice(len(pts), size=min(cnt, len(pts)), replace=False))] if len(pts) else pts
            E = np.concatenate([E, draw(5), E[:3]]) if len(E) else draw(5)  # absent + duplicates
            say(f"step {step}: erase {len(E)}")
            ne_g = G.erase(to_dev(E, dev))
            ne_m = M.erase(E)
            assert ne_g == ne_m, (ne_g, ne_m)
        same_state(G, M, f"step {step}")
        if M.size():
            q = draw(60)
            gi, gd = host(*G.knn(to_dev(q, dev), k))
            pts, ids = M.live()
            oi, od = oracle.knn_brute(pts, q, k, ids=ids, nthreads=8)
            if dtype == np.int32:
                assert_int_equal(gi, gd, oi, od)
            else:
                # map ids to rows of the live set for the distance recheck
                pos = {int(t): r for r, t in enumerate(ids.tolist())}
                gr = np.vectorize(lambda t: pos.get(int(t), -1))(gi)
                orr = np.vectorize(lambda t: pos.get(int(t), -1))(oi)
                assert_float_close(gr, gd, orr, od, pts, q)


def test_random_sequence_int_duplicates(pg, dev):
    _run_sequence(pg, dev, d=3, X=16, steps=30, coord_hi=10, dtype=np.int32, seed=1)


def test_random_sequence_int_wide(pg, dev):
    _run_sequence(pg, dev, d=2, X=64, steps=24, coord_hi=1 << 20, dtype=np.int32, seed=2, k=10)


def test_random_sequence_float(pg, dev):
    _run_sequence(pg, dev, d=3, X=32, steps=18, coord_hi=64, dtype=np.float32, seed=3)


def test_random_sequence_d5_leaf1(pg, dev):
    _run_sequence(pg, dev, d=5, X=4, steps=21, coord_hi=6, dtype=np.int32, seed=4, k=3, leaf=1)


@pytest.mark.parametrize("d,X,coord_hi,dtype,leaf,k", [(3, 16, 10, np.int32, 8, 7),
                                                     (2, 64, 1 << 20, np.int32, 16, 10),
                                                     (3, 32, 64, np.float32, 8, 7),
                                                     (5, 4, 6, np.int32, 1, 3)])
def test_random_sequence_spatial(pg, dev, d, X, coord_hi, dtype, leaf, k):
    # spatial-median static trees: same live set, so the same results
    _run_sequence(pg, dev, d=d, X=X, steps=18, coord_hi=coord_hi, dtype=dtype, seed=50 + d,
                  k=k, leaf=leaf, split="spatial")


@pytest.mark.parametrize("split", ["object", "spatial"])
def test_cfg5_shaped_reduced(pg, dev, split):
    """10% rounds as in the BDL experiments: 200k initial points, 3 rounds of
    20k inserts, 20k erases of live points, 20k fresh queries (k = 10)."""
    import torch
    init, rounds = datagen.bdl_rounds(200_000, 3, 20_000, 20_000, 3, seed=5)
    G = pg.BDLTree(3, torch.int32, leaf=16, X=1024, device=dev, split=split)
    M = BDLModel(3, 1024)
    G.insert(to_dev(init, dev))
    M.insert(init)
    same_state(G, M, "init")
    for r, rd in enumerate(rounds):
        say(f"round {r}")
        assert G.insert(to_dev(rd["insert"], dev)) == M.insert(rd["insert"])
        same_state(G, M, f"round {r} insert")
        pts, _ = M.live()
        E = datagen.choose_erase(pts, 20_000, rd["erase_seed"])
        assert G.erase(to_dev(E, dev)) == M.erase(E)
        same_state(G, M, f"round {r} erase")
        q = rd["queries"]
        gi, gd = host(*G.knn(to_dev(q, dev), 10))
        pts, ids = M.live()
        t = oracle.KdTree(pts, leaf=16)
        oi, od, _ = t.knn(q, 10, ids=ids)
        assert_int_equal(gi, gd, oi, od)


def test_cfg5_full_size(pg, dev):
    """The benchmarked batch-dynamic configuration: 10M initial points, 10
    rounds of 1M inserts, 1M erases of live points, 1M queries (k = 10).
    After every insert and every erase: F, buffer size, per-tree live counts
    and erase counts equal the model's (Algorithms 3 and 4); every query row
    byte-identical to the oracle's kd-tree search over the live set."""
    import torch
    init, rounds = datagen.bdl_rounds(10_000_000, 10, 1_000_000, 1_000_000, 3, seed=5)
    X = 1 << 14
    G = pg.BDLTree(3, torch.int32, leaf=16, X=X, device=dev)
    M = BDLModel(3, X)
    say("cfg5: initial insert")
    assert G.insert(to_dev(init, dev)) == M.insert(init) == 0
    same_state(G, M, "init")
    for r, rd in enumerate(rounds):
        say(f"cfg5 round {r}")
        assert G.insert(to_dev(rd["insert"], dev)) == M.insert(rd["insert"])
        same_state(G, M, f"round {r} insert")
        pts, _ = M.live()
        E = datagen.choose_erase(pts, 1_000_000, rd["erase_seed"])
        assert G.erase(to_dev(E, dev)) == M.erase(E)
        same_state(G, M, f"round {r} erase")
        gi, gd = host(*G.knn(to_dev(rd["queries"], dev), 10))
        pts, ids = M.live()
        oi, od, _ = oracle.KdTree(pts, leaf=16).knn(rd["queries"], 10, ids=ids, nthreads=16)
        assert_int_equal(gi, gd, oi, od)
