"""Pins for the oracle's BDL-tree model (Section 5, Appendix C Algorithms 3
and 4): the paper's worked insertion example, count invariants, and the
live set against an independent set computation."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.bdl_model import BDLModel, insert_plan

GOLD = os.path.join(os.path.dirname(__file__), "golden", "bdl_insert_example.json")


def _size(expr, X):
    return eval(expr, {"X": X})  # "X", "X+1", "X-1" from the fixture


@pytest.mark.parametrize("X", [3, 4, 8, 1000])
def test_paper_insert_example_planner(X):
    gold = json.load(open(GOLD))
    F, b = gold["start"]["F"], gold["start"]["buffer"]
    for st in gold["steps"]:
        p = insert_plan(F, b, _size(st["insert"], X), X)
        assert p["F_new"] == st["F"]
        assert p["buffer_after"] == st["buffer"]
        assert [i for i in range(8) if (p["destroyed"] >> i) & 1] == st["destroyed"]
        assert [i for i in range(8) if (p["new"] >> i) & 1] == st["built"]
        F, b = p["F_new"], p["buffer_after"]


@pytest.mark.parametrize("X", [3, 8])
def test_paper_insert_example_model(X):
    gold = json.load(open(GOLD))
    g = np.random.default_rng(X)
    M = BDLModel(2, X)
    M.insert(g.integers(0, 100, size=(_size(gold["start"]["points"], X), 2)).astype(np.int32))
    assert M.stats()[:2] == (gold["start"]["F"], gold["start"]["buffer"])
    for st in gold["steps"]:
        M.insert(g.integers(0, 100, size=(_size(st["insert"], X), 2)).astype(np.int32))
        F, b, live = M.stats()
        assert (F, b) == (st["F"], st["buffer"])
        for i in range(8):
            assert live[i] == ((X << i) if (F >> i) & 1 else 0)  # full trees


def test_planner_counts_random():
    g = np.random.default_rng(1)
    for X in (1, 2, 5, 64):
        F, b, total = 0, 0, 0
        sizes = {}
        for _ in range(200):
            m = int(g.integers(0, 5 * X + 3))
            p = insert_plan(F, b, m, X)
            for i in range(64):
                if (p["destroyed"] >> i) & 1:
                    sizes.pop(i)
            for j, q in p["quota"].items():
                sizes[j] = q + sum((X << i) for i in p["assign"].get(j, []))
                assert sizes[j] == X << j
            F, b, total = p["F_new"], p["buffer_after"], total + m
            assert 0 <= b < X
            assert sum(sizes.values()) + b == total
            assert F == sum(1 << i for i in sizes)


def test_model_live_set_and_knn():
    g = np.random.default_rng(3)
    d, X = 3, 16
    M = BDLModel(d, X)
    rows, alive = [], []
    for step in range(30):
        if step % 3 != 2:
            P = g.integers(0, 12, size=(int(g.integers(0, 90)), d)).astype(np.int32)
            first = M.insert(P)
            assert first == len(rows)
            rows += [tuple(r) for r in P.tolist()]
            alive += [True] * len(P)
        else:
            live_rows = [i for i, a in enumerate(alive) if a]
            pick = g.choice(len(live_rows), size=min(25, len(live_rows)), replace=False) if live_rows else []
            E = np.array([rows[live_rows[i]] for i in pick] + [(99, 99, 99)], dtype=np.int32).reshape(-1, d)
            want = {tuple(e) for e in E.tolist()}
            expect = sum(1 for i, a in enumerate(alive) if a and rows[i] in want)
            for i, a in enumerate(alive):
                if a and rows[i] in want:
                    alive[i] = False
            assert M.erase(E) == expect
        F, b, live = M.stats()
        assert 0 <= b < X
        assert sum(live) + b == sum(alive) == M.size()
        for i in range(64):
            if (F >> i) & 1:
                assert 2 * live[i] >= (X << i) or step % 3 != 2
                assert live[i] <= X << i
        pts, ids = M.live()
        assert ids.tolist() == [i for i, a in enumerate(alive) if a]
        if len(pts):
            q = g.integers(0, 12, size=(20, d)).astype(np.int32)
            a_ids, a_d = oracle.knn_brute(pts, q, 6, ids=ids)
            t = oracle.KdTree(pts, leaf=4)
            b_ids, b_d, _ = t.knn(q, 6, ids=ids)
            assert np.array_equal(a_ids, b_ids) and np.array_equal(a_d, b_d)
