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


def test_build_bytes_model():
    # ingest n(4d + 4(d+1)) + L levels of n(4 + 8(d+1)): 748 B per point at
    # d = 3, L = 20 (the headline tree)
    assert bench.tree_levels(10_000_000) == 20
    assert bench.build_bytes(10_000_000, 3, 20) == 748 * 10_000_000
    assert bench.tree_levels(16) == 0 and bench.tree_levels(17) == 1


def test_other_visit_constants_match_the_oracle():
    """The visit counts behind the other k-NN rooflines, from fresh samples:
    5-D clustered queries, fresh uniform queries over 10M points, and the
    sphere clouds (other clouds than the constants were drawn from)."""
    f, q = datagen.clustered(bench.N, 5, seed=3, n_queries=1_000_000, query_seed=33)
    rows = np.random.default_rng(22).choice(len(q), 20_000, replace=False)
    _, _, c = oracle.KdTree(f, leaf=16).knn(q[rows], 5, nthreads=8)
    vi, vp = bench.VISITS["clustered_5d_queries"]
    assert c[0] / len(rows) == pytest.approx(vi, rel=0.03)
    assert c[2] / len(rows) == pytest.approx(vp, rel=0.03)
    del f, q
    init, rounds = datagen.bdl_rounds(bench.N, 1, 1_000_000, 1_000_000, 3, seed=5)
    rows = np.random.default_rng(23).choice(1_000_000, 20_000, replace=False)
    _, _, c = oracle.KdTree(init, leaf=16).knn(rounds[0]["queries"][rows], 10, nthreads=8)
    vi, vp = bench.VISITS["uniform_3d_fresh_queries"]
    assert c[0] / len(rows) == pytest.approx(vi, rel=0.01)
    assert c[2] / len(rows) == pytest.approx(vp, rel=0.01)
    from oracle.visit_counts import cloud_counts
    cc = cloud_counts(16, 16, stride=16, offset=8)  # the interleaved other stratum
    vi, vp = bench.VISITS["sphere_clouds_all_points"]
    assert cc["n_int"] == pytest.approx(vi, rel=0.02)
    assert cc["n_pts"] == pytest.approx(vp, rel=0.02)


def test_bdl_byte_models():
    # one new tree of 16384 * 2^6 points and a rebuilt buffer of 576, one
    # destroyed tree of 16384 * 2^5 live points
    X = 1 << 14
    before = (1 << 5, 100, [0] * 5 + [X << 5] + [0] * 34)
    after = (1 << 6, 576, [0] * 6 + [X << 6] + [0] * 33)
    m = 1_000_000
    want = (m * 12 + bench.build_bytes(X << 6, 3, bench.tree_levels(X << 6))
            + (X << 5) * (16 + 12 + 8) + bench.build_bytes(576, 3, bench.tree_levels(576)))
    assert bench.bdl_insert_bytes(before, after, m) == want
    # erase: per point 12 + per tree (4 L + 16 n / 2^L)
    n = X << 6
    L = bench.tree_levels(n)
    assert bench.bdl_erase_bytes(after, 10) == pytest.approx(
        10 * (12 + 4 * L + 16 * n / (1 << L) + 4 * bench.tree_levels(576) + 16 * 576 / (1 << bench.tree_levels(576))))
