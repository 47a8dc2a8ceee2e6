"""Per-query visit counts of the oracle's kd-tree k-NN search (Appendix C,
"Data-Parallel k-NN") on a seeded sample -- the figures behind the
algorithmic byte model of the k-NN kernel:

    bytes/query = 4 d                (query coordinates)
                + k (4 + s)          (output row; s = 8 int64 / 4 float32)
                + 4 N_int            (split values of visited internal nodes)
                + 4 (d + 1) N_pts    (coordinates + index of scanned points)

Run:  python -m oracle.visit_counts [n] [d] [k] [leaf] [sample]
(defaults: the 3-D, n = 10M, k = 10, leaf 16 all-points workload, 100,000
sampled queries), or  python -m oracle.visit_counts --workloads  for the
counts of every benchmarked search (the headline all-points search, the
5-D clustered queries, fresh uniform queries of the batch-dynamic rounds,
and all-points searches within the sphere clouds).  TEST INFRASTRUCTURE:
calls only the oracle.
"""
import sys
import time

import numpy as np

import oracle
from paper_2207_01834_amd import datagen


def counts(points, k, leaf, sample, seed=0):
    t0 = time.perf_counter()
    t = oracle.KdTree(points, leaf=leaf)
    tb = time.perf_counter() - t0
    rows = np.random.default_rng(seed).choice(len(points), size=min(sample, len(points)), replace=False)
    t0 = time.perf_counter()
    _, _, c = t.knn(points[rows], k)
    tq = time.perf_counter() - t0
    m = len(rows)
    return {"n_int": c[0] / m, "n_leaves": c[1] / m, "n_pts": c[2] / m,
            "build_s": tb, "query_s": tq, "sample": m}


def query_counts(points, queries, k, leaf, sample, seed=0):
    """Visit counts of a sample of a separate query set."""
    t = oracle.KdTree(points, leaf=leaf)
    rows = np.random.default_rng(seed).choice(len(queries), size=min(sample, len(queries)),
                                              replace=False)
    _, _, c = t.knn(queries[rows], k, nthreads=8)
    m = len(rows)
    return {"n_int": c[0] / m, "n_leaves": c[1] / m, "n_pts": c[2] / m, "sample": m}


def cloud_counts(k, leaf, stride=16, offset=0):
    """Per-point visit counts of all-points searches within the 4,096 sphere
    clouds: every point of a stratified sample of clouds (in size order,
    every stride-th from offset), weighted by cloud size (an estimate of the
    mean over all points of the batch)."""
    sizes = datagen.cloud_sizes(4096, seed=4)
    pts, offs = datagen.sphere_clouds(sizes, seed=44)
    pick = np.argsort(sizes, kind="stable")[offset::stride]
    n_clouds = len(pick)
    tot = np.zeros(3)
    w = 0
    for c in pick:
        cloud = pts[offs[c]:offs[c + 1]]
        _, _, cnt = oracle.KdTree(cloud, leaf=leaf).knn(cloud, k, nthreads=8)
        tot += cnt
        w += len(cloud)
    # size-weighted: sum of counts / sum of points over the drawn clouds
    return {"n_int": tot[0] / w, "n_leaves": tot[1] / w, "n_pts": tot[2] / w, "clouds": n_clouds,
            "points": int(w)}


def workloads():
    out = {}
    pts = datagen.uniform_int(10_000_000, 3, seed=2)
    out["headline_all_points_3d"] = counts(pts, 10, 16, 100_000)
    f, q = datagen.clustered(10_000_000, 5, seed=3, n_queries=1_000_000, query_seed=33)
    out["clustered_5d_queries"] = query_counts(f, q, 5, 16, 100_000)
    init, rounds = datagen.bdl_rounds(10_000_000, 1, 1_000_000, 1_000_000, 3, seed=5)
    out["uniform_3d_fresh_queries"] = query_counts(init, rounds[0]["queries"], 10, 16, 100_000)
    out["sphere_clouds_all_points"] = cloud_counts(16, 16, 16, 0)
    return out


def bytes_per_query(d, k, dist_bytes, n_int, n_pts):
    return 4 * d + k * (4 + dist_bytes) + 4 * n_int + 4 * (d + 1) * n_pts


if __name__ == "__main__":
    if sys.argv[1:] == ["--workloads"]:
        for name, c in workloads().items():
            print(name, {k: (round(v, 3) if isinstance(v, float) else v) for k, v in c.items()})
        sys.exit(0)
    a = [int(x) for x in sys.argv[1:]]
    n, d, k, leaf, sample = (a + [10_000_000, 3, 10, 16, 100_000][len(a):])[:5]
    pts = datagen.uniform_int(n, d, seed=2)
    c = counts(pts, k, leaf, sample)
    c["bytes_per_query_int"] = bytes_per_query(d, k, 8, c["n_int"], c["n_pts"])
    c["bytes_per_query_float"] = bytes_per_query(d, k, 4, c["n_int"], c["n_pts"])
    for key, v in c.items():
        print(f"{key}: {v:.3f}" if isinstance(v, float) else f"{key}: {v}")
