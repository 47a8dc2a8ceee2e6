"""Per-query visit counts of the oracle's kd-tree k-NN search (Appendix C,
"Data-Parallel k-NN") on a seeded sample -- the figures behind the
algorithmic byte model of the k-NN kernel:

    bytes/query = 4 d                (query coordinates)
                + k (4 + s)          (output row; s = 8 int64 / 4 float32)
                + 4 N_int            (split values of visited internal nodes)
                + 4 (d + 1) N_pts    (coordinates + index of scanned points)

Run:  python -m oracle.visit_counts [n] [d] [k] [leaf] [sample]
(defaults: the 3-D, n = 10M, k = 10, leaf 16 all-points workload, 100,000
sampled queries).  TEST INFRASTRUCTURE: calls only the oracle.
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


def bytes_per_query(d, k, dist_bytes, n_int, n_pts):
    return 4 * d + k * (4 + dist_bytes) + 4 * n_int + 4 * (d + 1) * n_pts


if __name__ == "__main__":
    a = [int(x) for x in sys.argv[1:]]
    n, d, k, leaf, sample = (a + [10_000_000, 3, 10, 16, 100_000][len(a):])[:5]
    pts = datagen.uniform_int(n, d, seed=2)
    c = counts(pts, k, leaf, sample)
    c["bytes_per_query_int"] = bytes_per_query(d, k, 8, c["n_int"], c["n_pts"])
    c["bytes_per_query_float"] = bytes_per_query(d, k, 4, c["n_int"], c["n_pts"])
    for key, v in c.items():
        print(f"{key}: {v:.3f}" if isinstance(v, float) else f"{key}: {v}")
