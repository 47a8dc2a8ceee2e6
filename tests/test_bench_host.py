"""Host-side arithmetic of bench.py: the algorithmic bytes behind the
roofline line are pinned to the oracle's own visit counts on the headline
workload, and the counter-to-traffic scaling is checked on synthetic
counter files."""
import csv
import json

import numpy as np
import pytest

import bench
import oracle
from paper_2207_01834_amd import datagen


def test_bytes_per_query_formula():
    # 4d (query) + k(4 + s) (output) + 4 N_int (split values) + 4(d+1) N_pts (records)
    d, k = bench.D, bench.K
    for s in (8, 4):
        want = 4 * d + k * (4 + s) + 4 * bench.N_INT + 4 * (d + 1) * bench.N_PTS
        assert bench.bytes_per_query(s) == pytest.approx(want)
    assert bench.bytes_per_query(8) == pytest.approx(1776.892, abs=1e-3)


def test_visit_constants_match_the_oracle():
    """N_INT and N_PTS are the oracle search's mean visits per query on the
    headline points (10M uniform 3-D, leaf 16, k = 10); a fresh sample must
    agree within sampling noise."""
    pts = datagen.uniform_int(bench.N, bench.D, seed=2)
    t = oracle.KdTree(pts, leaf=bench.LEAF)
    rows = np.random.default_rng(21).choice(len(pts), 20_000, replace=False)
    _, _, cnt = t.knn(pts[rows], bench.K)
    assert cnt[0] / len(rows) == pytest.approx(bench.N_INT, rel=0.01)
    assert cnt[2] / len(rows) == pytest.approx(bench.N_PTS, rel=0.01)


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": v})


def test_write_traffic_scaling(tmp_path):
    # the copy probe moves 1024 MiB each way; its counters read 2x (fetch)
    # and 0.5x (write) of that, so the k-NN counters are scaled by 1/2 and 2
    mib = 1024
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    knn = "void pg::knn_detail::knn_static_kernel<int, 3, 10, true, false, false>"
    _counter_csv(f, [(knn, 3000.0), (knn, 3100.0), (knn, 2900.0)] +
                 [("__amd_rocclr_copyBuffer", 2 * mib * 1024.0)] * 3 + [("__amd_rocclr_copyBuffer", 4.0)])
    _counter_csv(w, [(knn, 1000.0)] * 3 + [("__amd_rocclr_copyBuffer", 0.5 * mib * 1024.0)] * 3)
    out = tmp_path / "t.json"
    rec = bench.write_traffic(str(f), str(w), "int", mib, "cmd", out_path=str(out))
    assert rec["fetch_scale"] == pytest.approx(0.5) and rec["write_scale"] == pytest.approx(2.0)
    assert rec["hbm_bytes_per_launch"] == pytest.approx((3000.0 * 0.5 + 1000.0 * 2.0) * 1024.0)
    assert json.loads(out.read_text())["source_hash"] == bench.knn_source_hash()


def test_range_bytes_formula():
    d = 2
    tree = 8 * d + 8 * d * bench.R_NODES + 4 * (d + 1) * bench.R_PTS
    assert bench.range_bytes_per_query(d, 10.5, False) == pytest.approx(tree + 4)
    assert bench.range_bytes_per_query(d, 10.5, True) == pytest.approx(tree + 8 + 42)


def test_range_constants_match_the_oracle():
    """R_NODES and R_PTS are the oracle tree search's node boxes and points
    tested per query on the 2-D range workload (10M uniform points, a square
    of half side 512 around every point, leaf 16)."""
    pts = datagen.uniform_int(bench.N, 2, seed=2)
    t = oracle.KdTree(pts, leaf=bench.LEAF)
    rows = np.random.default_rng(22).choice(len(pts), 20_000, replace=False)
    boxes = datagen.range_boxes(pts[rows], 512)
    *_, cnt = t.range(boxes)
    assert cnt[0] / len(rows) == pytest.approx(bench.R_NODES, rel=0.01)
    assert cnt[1] / len(rows) == pytest.approx(bench.R_PTS, rel=0.01)
