#!/usr/bin/env python3
"""Benchmark: static 3-D kd-tree build + all-points k-NN on one MI355X.

Workload (the paper's uniform data set shape, Section 6): n = 10,000,000
points with int32 coordinates uniform in [0, 2^20)^3 (seed 2), k = 10,
leaves of at most 16 points, every point queried.  One step = build the tree
from device-resident points + k-NN of all n points.  ``value`` is the
end-to-end rate (queries per second of the whole step, build included);
``build_mpts_s`` and ``knn_qps`` give the two parts.

The roofline object covers the dominant kernel (the k-NN search): its
algorithmic bytes per query, 4d + k(4 + 8) + 4 N_int + 4(d+1) N_pts, take
the internal nodes and points the oracle's canonical search visits per query
on this workload (``python -m oracle.visit_counts``), are multiplied by the n
queries of one launch and divided by the launch time measured with HIP events
on the stream the kernel runs on.  ``traffic`` is the HBM bytes the kernel
really moved, from rocprofv3 counters (``--write-traffic``).

The cpu_baseline object times the CPU oracle (serial C) on the same points:
the full tree build and the k-NN search of a sample of queries, projected to
the whole step.

Progress goes to stderr; stdout carries exactly one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N, D, K, LEAF = 10_000_000, 3, 10, 16

# Oracle visit counts per query on this workload (100,000 sampled queries):
# internal nodes 40.923, points 92.575  ->  bytes/query = 4d + k(4+s) + 4 N_int
# + 4(d+1) N_pts with s = 8 (int64 distances) or 4 (float32 distances).
N_INT, N_PTS = 40.923, 92.575


def bytes_per_query(dist_bytes):
    return 4 * D + K * (4 + dist_bytes) + 4 * N_INT + 4 * (D + 1) * N_PTS


# Oracle visit counts (internal nodes, points) per query of the other
# benchmarked searches (``python -m oracle.visit_counts --workloads``):
# 5-D clustered queries (k = 5), fresh uniform 3-D queries of the
# batch-dynamic rounds over 10M points (k = 10), all-points searches within
# the sphere clouds (k = 16, size-weighted over every 16th cloud in size
# order: 256 clouds, 3.07M points).
VISITS = {
    "clustered_5d_queries": (115.277, 332.081),
    "uniform_3d_fresh_queries": (41.89, 96.63),
    "sphere_clouds_all_points": (21.653, 83.576),
}


def knn_bytes(d, k, id_bytes, dist_bytes, n_int, n_pts):
    """Algorithmic bytes of one k-NN query: the query, its output row, the
    split values of the visited internal nodes and the records of the
    scanned points (the oracle's visits)."""
    return 4 * d + k * (id_bytes + dist_bytes) + 4 * n_int + 4 * (d + 1) * n_pts


def build_bytes(n, d, L):
    """Algorithmic bytes of the object-median build the paper describes as
    O(n) per level: ingest (rows read, key planes and rows written) plus, per
    level, one key read and one record read and write."""
    return n * (4 * d + 4 * (d + 1)) + L * n * (4 + 8 * (d + 1))


def tree_levels(n, leaf=16):
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    return L


def roof(nbytes, ms, kernel, model):
    """Roofline object of one timed call: algorithmic bytes over its time
    against the HBM peak."""
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": nbytes,
            "model": model}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def knn_source_hash():
    h = hashlib.sha256()
    for f in ("knn.hip", "knn_static.hpp", "knn_wave.hpp", "knn_int.hip", "search.hpp", "xsearch.hpp",
              "knn.hpp", "common.hpp", "wave.hpp"):
        with open(os.path.join(ROOT, "paper_2207_01834_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(dtype):
    """HBM bytes per k-NN launch from the committed rocprofv3 counter summary,
    when it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"knn_all_{dtype}3d_10M_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != knn_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def write_traffic(fetch_csv, write_csv, dtype, mib, command, out_path=None):
    """Turns two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) of a bench run with the copy probe into the traffic summary the
    roofline line reads.  Each counter is scaled by what it reads for the
    probe's device copy, which moves `mib` MiB in and `mib` MiB out."""
    import csv
    import statistics

    def per_kernel(path):
        rows = list(csv.DictReader(open(path)))
        knn = [float(r["Counter_Value"]) for r in rows if "knn_static_kernel" in r["Kernel_Name"]]
        cp = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        return knn, cp

    fk, fc = per_kernel(fetch_csv)
    wk, wc = per_kernel(write_csv)
    want = mib * 1024.0  # KiB each way
    # the probe's copies are the largest copy dispatches
    fc = sorted(fc)[-5:]
    wc = sorted(wc)[-5:]
    f_scale = want / statistics.median(fc)
    w_scale = want / statistics.median(wc)
    f_kib, w_kib = statistics.median(fk), statistics.median(wk)
    rec = {
        "kernel": "knn_static_kernel (all-points)",
        "workload": f"3-D n=10M {dtype} uniform, k=10, leaf 16",
        "fetch_kib_per_launch": f_kib, "write_kib_per_launch": w_kib,
        "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
        "copy_probe_mib": mib,
        "hbm_bytes_per_launch": (f_kib * f_scale + w_kib * w_scale) * 1024.0,
        "source_hash": knn_source_hash(),
        "command": command,
    }
    path = out_path or os.path.join(ROOT, "profiles", f"knn_all_{dtype}3d_10M_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))
    return rec


def copy_probe(torch, dev, mib):
    """Plain device-to-device copy of `mib` MiB: the achievable HBM rate in
    this run, and a kernel of known traffic for scaling counter readings."""
    if mib <= 0:
        return None
    n = mib * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.int32, device=dev).fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    return 2.0 * mib * (1 << 20) / (ms * 1e-3) / 1e9


def cpu_baseline(pts, sample):
    import numpy as np

    import oracle
    log(f"cpu baseline: oracle build of {len(pts)} points + {sample} sampled queries")
    t0 = time.perf_counter()
    t = oracle.KdTree(pts, leaf=LEAF)
    tb = time.perf_counter() - t0
    rows = np.random.default_rng(7).choice(len(pts), size=sample, replace=False)
    t0 = time.perf_counter()
    _, _, cnt = t.knn(pts[rows], K)
    tq = time.perf_counter() - t0
    step_s = tb + tq * len(pts) / sample
    # the same search, query-parallel: static chunks over every core this
    # process may run on (the C call releases the interpreter lock)
    from concurrent.futures import ThreadPoolExecutor
    threads = min(len(os.sched_getaffinity(0)), 16)
    psample = min(len(pts), sample * threads)
    prow = np.random.default_rng(8).choice(len(pts), size=psample, replace=False)
    chunks = np.array_split(pts[prow], threads)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda c: t.knn(c, K), chunks))
    tp = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": len(pts) / step_s, "unit": "queries/s", "cores": 1, "kind": "oracle",
        "sample": (f"serial C oracle: full object-median build of all {len(pts):,} points "
                   f"({tb:.2f} s) + kd-tree k-NN of {sample:,} sampled points ({tq:.2f} s), "
                   f"projected to the {len(pts):,}-query step"),
        "build_mpts_s": len(pts) / tb / 1e6, "knn_qps": sample / tq,
        "visits_per_query": {"internal": cnt[0] / sample, "leaves": cnt[1] / sample,
                             "points": cnt[2] / sample},
        "query_parallel": {"threads": threads, "cpu": model, "queries": psample,
                           "knn_qps": psample / tp,
                           "step_qps": len(pts) / (tb + tp * len(pts) / psample),
                           "note": "k-NN in static chunks on one thread per core; the build "
                                   "stays serial"},
    }


def timed(torch, fn, reps=3):
    """Median milliseconds of fn() over reps runs (HIP events on the current
    stream, which the library launches on)."""
    import numpy as np
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return float(np.median(out))


def form_static_float(torch, pg, datagen, dev):
    """The same workload with float32 coordinates (int grid / 2^20)."""
    pts = datagen.int_to_unit_float(datagen.uniform_int(N, D, seed=2))
    x = torch.from_numpy(pts).to(dev)
    idx = torch.empty((N, K), dtype=torch.int32, device=dev)
    dist = torch.empty((N, K), dtype=torch.float32, device=dev)
    holder = {}
    build_ms = timed(torch, lambda: holder.__setitem__("t", pg.kdtree_build(x, leaf=LEAF)))
    knn_ms = timed(torch, lambda: holder["t"].knn_all(K, out=(idx, dist)))
    return {"workload": "3-D n=10M float32 uniform, k=10, leaf 16, all points",
            "build_ms": build_ms, "knn_ms": knn_ms, "knn_qps": N / (knn_ms * 1e-3),
            "build_mpts_s": N / (build_ms * 1e-3) / 1e6,
            "roofline": roof(bytes_per_query(4) * N, knn_ms, "knn_static_kernel (all-points)",
                             "headline visit counts, float32 distances"),
            "build_roofline": roof(build_bytes(N, D, tree_levels(N)), build_ms, "build (all kernels)",
                                   "n(8d+4) + L n (8d+12)")}


def form_graph(torch, pg, datagen, dev):
    """k-NN graph on the headline points (3-D 10M int uniform, k = 10, leaf
    16): each point's 10 nearest other points, from a built tree."""
    pts = datagen.uniform_int(N, D, seed=2)
    x = torch.from_numpy(pts).to(dev)
    t = pg.kdtree_build(x, leaf=LEAF)
    idx = torch.empty((N, K), dtype=torch.int32, device=dev)
    dist = torch.empty((N, K), dtype=torch.int64, device=dev)
    graph_ms = timed(torch, lambda: t.knn_graph(K, out=(idx, dist)))
    return {"workload": "k-NN graph, 3-D n=10M int32 uniform, k=10 other points per point, leaf 16",
            "graph_ms": graph_ms, "edges_per_s": N * K / (graph_ms * 1e-3),
            "roofline": roof(bytes_per_query(8) * N, graph_ms, "knn_static_kernel (all-points, own "
                             "point excluded)", "headline visit counts")}


def form_spatial(torch, pg, datagen, dev):
    """Spatial-median splits down to at most 16 points per leaf, each node
    cutting its cell or the bounding box of its own points, on the headline
    points and on the 5-D clustered set: build and k-NN beside the
    object-median numbers of the other forms."""
    import numpy as np
    out = {}
    pts = datagen.uniform_int(N, D, seed=2)
    x = torch.from_numpy(pts).to(dev)
    idx = torch.empty((N, K), dtype=torch.int32, device=dev)
    dist = torch.empty((N, K), dtype=torch.int64, device=dev)
    holder = {}
    for space, tag in (("cell", ""), ("points", "_point_box")):
        b_ms = timed(torch, lambda: holder.__setitem__(
            "t", pg.kdtree_build(x, leaf=LEAF, split="spatial", space=space)))
        t = holder["t"]
        k_ms = timed(torch, lambda: t.knn_all(K, out=(idx, dist)))
        sizes = np.diff(t.offsets())
        nodes, leaves = t.counts()
        out["uniform_3d" + tag] = {"workload": f"3-D n=10M int32 uniform, k=10, leaf 16, all points, "
                                               f"nodes cut their {space if space == 'cell' else 'point box'}",
                                   "build_ms": b_ms, "knn_ms": k_ms, "max_leaf": int(sizes.max()),
                                   "empty_leaves": int((sizes == 0).sum()), "nodes": nodes,
                                   "levels": t.levels,
                                   "roofline": roof(bytes_per_query(8) * N, k_ms,
                                                    "knn_static_kernel (explicit-node walk)",
                                                    "the object-median search's visit counts (the "
                                                    "algorithm's bytes, not this tree's)")}
        del t, holder["t"]
    del idx, dist, x
    f, q = datagen.clustered(N, 5, seed=3, n_queries=1_000_000, query_seed=33)
    xf = torch.from_numpy(f).to(dev)
    qd = torch.from_numpy(q).to(dev)
    for space, tag, reps in (("cell", "", 3), ("points", "_point_box", 3)):
        b_ms = timed(torch, lambda: holder.__setitem__(
            "t", pg.kdtree_build(xf, leaf=LEAF, split="spatial", space=space)))
        t = holder["t"]
        k_ms = timed(torch, lambda: t.knn(qd, 5), reps=reps)
        sizes = np.diff(t.offsets())
        nodes, leaves = t.counts()
        vi, vp = VISITS["clustered_5d_queries"]
        out["clustered_5d" + tag] = {"workload": f"5-D n=10M clustered float32, 1M queries, k=5, leaf 16, "
                                                 f"nodes cut their {space if space == 'cell' else 'point box'}",
                                     "build_ms": b_ms, "knn_ms": k_ms, "max_leaf": int(sizes.max()),
                                     "empty_leaves": int((sizes == 0).sum()), "nodes": nodes,
                                     "levels": t.levels,
                                     "roofline": roof(knn_bytes(5, 5, 4, 4, vi, vp) * len(q), k_ms,
                                                      "knn_static_kernel (explicit-node walk)",
                                                      "the object-median search's visit counts")}
        del t, holder["t"]
    return out


def form_clustered(torch, pg, datagen, dev):
    """5-D clustered float32 (1,000 Gaussian clusters, Zipf sizes), 1M queries
    from the same mixture, k = 5."""
    pts, q = datagen.clustered(N, 5, seed=3, n_queries=1_000_000, query_seed=33)
    x = torch.from_numpy(pts).to(dev)
    qd = torch.from_numpy(q).to(dev)
    holder = {}
    build_ms = timed(torch, lambda: holder.__setitem__("t", pg.kdtree_build(x, leaf=LEAF)))
    knn_ms = timed(torch, lambda: holder["t"].knn(qd, 5))
    vi, vp = VISITS["clustered_5d_queries"]
    return {"workload": "5-D n=10M clustered float32, 1M queries, k=5, leaf 16",
            "build_ms": build_ms, "knn_ms": knn_ms, "knn_qps": len(q) / (knn_ms * 1e-3),
            "build_mpts_s": N / (build_ms * 1e-3) / 1e6,
            "roofline": roof(knn_bytes(5, 5, 4, 4, vi, vp) * len(q), knn_ms,
                             "knn_static_kernel (queries ordered by leaf)",
                             f"oracle visits {vi} internal nodes, {vp} points per query"),
            "build_roofline": roof(build_bytes(N, 5, tree_levels(N)), build_ms, "build (all kernels)",
                                   "n(8d+4) + L n (8d+12)")}


def bdl_insert_bytes(before, after, m, d=3, X=1 << 14):
    """Algorithmic bytes of one BDL insert from the forest before and after
    it (F, buffer size, live points per tree): the batch read, the live
    points of destroyed trees gathered (read 4(d+1), written 4d + 8), and
    every new tree and the new buffer built (build_bytes)."""
    F0, b0, live0 = before
    F1, b1, live1 = after
    nb = m * 4 * d
    for i in range(len(live1)):
        if (F1 >> i) & 1 and not (F0 >> i) & 1:
            nb += build_bytes(live1[i], d, tree_levels(live1[i]))
        if (F0 >> i) & 1 and not (F1 >> i) & 1:
            nb += live0[i] * (4 * (d + 1) + 4 * d + 8)
    if b1 != b0 or F1 != F0:
        nb += build_bytes(b1, d, tree_levels(b1))
    return nb


def bdl_erase_bytes(state, m, d=3):
    """Algorithmic bytes of one erase batch of m points: each point read,
    and in every tree of the forest one descent (a split value per level)
    and one leaf scanned (its records)."""
    F, b, live = state
    per = 4 * d
    for n_t in [live[i] for i in range(len(live)) if (F >> i) & 1] + ([b] if b else []):
        L = tree_levels(n_t)
        per += 4 * L + 4 * (d + 1) * n_t / (1 << L)
    return m * per


def form_bdl(torch, pg, datagen, dev, rounds, with_oracle=False):
    """Batch-dynamic: 10M initial 3-D int points, then rounds of 1M inserts,
    1M erases of live points, 1M fresh queries (k = 10), X = 2^14.  With
    the oracle: the serial C oracle's time for the last round's queries (a
    tree over the live points, 10,000 sampled queries projected to 1M)."""
    import numpy as np
    init, rds = datagen.bdl_rounds(N, rounds, 1_000_000, 1_000_000, 3, seed=5)
    warm_dynamic(torch, pg, datagen, 3, dev)
    B = pg.BDLTree(3, torch.int32, leaf=LEAF, X=1 << 14, device=dev)
    xi = torch.from_numpy(init).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.insert(xi)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    pool = init
    ins, era, knn = [], [], []
    ins_b, era_b = [], []
    erased_total = 0
    for r, rd in enumerate(rds):
        xr = torch.from_numpy(rd["insert"]).to(dev)
        before = B.stats(40)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.insert(xr)
        torch.cuda.synchronize()
        ins.append((time.perf_counter() - t0) * 1e3)
        after = B.stats(40)
        ins_b.append(bdl_insert_bytes(before, after, len(rd["insert"])))
        era_b.append(bdl_erase_bytes(after, 1_000_000))
        pool = np.concatenate([pool, rd["insert"]])
        g = np.random.default_rng(rd["erase_seed"])
        pick = g.choice(len(pool), size=1_000_000, replace=False)
        E = torch.from_numpy(np.ascontiguousarray(pool[pick])).to(dev)
        keep = np.ones(len(pool), bool)
        keep[pick] = False
        pool = pool[keep]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        erased_total += B.erase(E)
        torch.cuda.synchronize()
        era.append((time.perf_counter() - t0) * 1e3)
        qd = torch.from_numpy(rd["queries"]).to(dev)
        knn.append(timed(torch, lambda: B.knn(qd, 10), reps=1))
    med = lambda a: float(np.median(a))
    vi, vp = VISITS["uniform_3d_fresh_queries"]
    # per-round algorithmic bytes over per-round time, median over rounds
    ins_gbs = [b / (t * 1e-3) / 1e9 for b, t in zip(ins_b, ins)]
    era_gbs = [b / (t * 1e-3) / 1e9 for b, t in zip(era_b, era)]
    knn_bytes_1m = knn_bytes(3, 10, 8, 8, vi, vp) * 1e6
    out = {"workload": "BDL 3-D int, 10M initial, rounds of 1M insert / 1M erase / 1M kNN (k=10), X=2^14",
           "rounds": rounds, "initial_insert_ms": build_ms,
           "insert_ms": med(ins), "erase_ms": med(era), "knn_ms": med(knn),
           "insert_mpts_s": 1.0 / med(ins) * 1e3, "erase_mpts_s": 1.0 / med(era) * 1e3,
           "knn_qps": 1e6 / (med(knn) * 1e-3), "erased_per_round": erased_total / rounds,
           "live_points": B.size(),
           "roofline": roof(knn_bytes_1m, med(knn), "bdl_knn_kernel (all trees, one k-list)",
                            f"one tree over the live set: {vi} internal nodes, {vp} points per "
                            "query (a forest visits more)"),
           "insert_roofline": roof(med(ins_b), med(ins), "insert (gather + builds)",
                                   "batch read + destroyed trees gathered + new trees and buffer "
                                   "built (build_bytes); wall time incl. host planning"),
           "erase_roofline": roof(med(era_b), med(era), "erase_kernel (one walk per point and tree)",
                                  "per point: its coordinates + per tree one descent and one leaf"),
           "insert_gbs_per_round": [round(v, 1) for v in ins_gbs],
           "erase_gbs_per_round": [round(v, 1) for v in era_gbs]}
    if with_oracle and rds:
        import oracle
        q = rds[-1]["queries"][:10_000]
        t0 = time.perf_counter()
        T = oracle.KdTree(pool, leaf=LEAF)
        tb = time.perf_counter() - t0
        t0 = time.perf_counter()
        T.knn(q, 10)
        tq = (time.perf_counter() - t0) * len(rds[-1]["queries"]) / len(q)
        out["oracle_round"] = {"cores": 1, "build_live_s": tb, "knn_1M_s_projected": tq,
                               "round_s": tb + tq,
                               "sample": "serial C oracle: one tree over the last round's live points, "
                                         "10,000 of its 1M queries, projected"}
    return out


def form_baselines(torch, pg, datagen, dev, rounds):
    """The two baselines of Section 6.3 on the BDL rounds (10M initial 3-D
    int points; per round 1M inserts, 1M erases of live points, 1M fresh
    queries, k = 10): B1 rebuilds one tree after every batch, B2 keeps its
    splits (inserts join leaves, erases leave tombstones).  Median per round."""
    import numpy as np
    init, rds = datagen.bdl_rounds(N, rounds, 1_000_000, 1_000_000, 3, seed=5)
    out = {"workload": f"10M initial 3-D int32 uniform points, {rounds} rounds of 1M insert / "
                       "1M erase / 1M k-NN (k=10), leaf 16"}
    for name in ("b1", "b2"):
        x = torch.from_numpy(init).to(dev)
        if name == "b1":
            G = pg.B1Tree(3, torch.int32, leaf=LEAF, device=dev)
            G.insert(x)
        else:
            G = pg.B2Tree(x, leaf=LEAF)
        pool = init
        ins, era, knn = [], [], []
        for rd in rds:  # the same batches as the BDL form
            P = torch.from_numpy(rd["insert"]).to(dev)
            ins.append(timed(torch, lambda: G.insert(P), reps=1))
            pool = np.concatenate([pool, rd["insert"]])
            g = np.random.default_rng(rd["erase_seed"])
            pick = g.choice(len(pool), size=1_000_000, replace=False)
            E = torch.from_numpy(np.ascontiguousarray(pool[pick])).to(dev)
            keep = np.ones(len(pool), bool)
            keep[pick] = False
            pool = pool[keep]
            era.append(timed(torch, lambda: G.erase(E), reps=1))
            Q = torch.from_numpy(rd["queries"]).to(dev)
            knn.append(timed(torch, lambda: G.knn(Q, 10), reps=1))
        # byte models at the rounds' typical sizes: n live points before a
        # round's insert, m per batch
        n0, m, d = len(init), 1_000_000, 3
        L = tree_levels(n0 + m)
        leaf_pts = (n0 + m) / (1 << L)
        gather = (4 * (d + 1) + 4 * d + 8)
        if name == "b1":
            ins_b = m * 4 * d + n0 * gather + build_bytes(n0 + m, d, L)
            era_b = m * (4 * d + 4 * L + 4 * (d + 1) * leaf_pts) + n0 * gather + build_bytes(n0, d,
                                                                                              tree_levels(n0))
            imodel = "batch read + live points gathered + one build of all live points"
            emodel = "one descent and leaf per point + gather + rebuild of the live points"
        else:
            Lb = tree_levels(n0)  # B2's splits come from the initial points
            ins_b = m * (4 * d + 4 * Lb) + (n0 + m) * (8 * (d + 1) + 16)
            era_b = m * (4 * d + 4 * Lb + 4 * (d + 1) * (n0 + m) / (1 << Lb))
            imodel = "new points read and descended + every point moved to the grown arrays"
            emodel = "one descent and leaf per point"
        vi, vp = VISITS["uniform_3d_fresh_queries"]
        out[name] = {"insert_ms": float(np.median(ins)), "erase_ms": float(np.median(era)),
                     "knn_ms": float(np.median(knn)), "knn_ms_last": knn[-1],
                     "roofline": roof(knn_bytes(3, 10, 8, 8, vi, vp) * 1e6, float(np.median(knn)),
                                      "bdl_knn_kernel (one tree)",
                                      "the oracle search's visits on one tree over the live set"),
                     "insert_roofline": roof(ins_b, float(np.median(ins)), "insert", imodel),
                     "erase_roofline": roof(era_b, float(np.median(era)), "erase", emodel)}
        del G
        torch.cuda.empty_cache()
    return out


def wall_ms(torch, fn):
    """Milliseconds of one fn() call between two device synchronisations
    (the update calls synchronise inside, so events would miss host work)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, r


def grow_tree(torch, pg, kind, d, chunks, dev, split="object"):
    """One tree of `kind` (bdl, b1, b2) grown from device batches in order;
    B2 is built over the first batch (its splits come from it).  Returns the
    tree and the milliseconds of each batch."""
    G, ms = None, []
    for c in chunks:
        if G is None and kind == "b2":
            t, G = wall_ms(torch, lambda: pg.B2Tree(c, leaf=LEAF, split=split))
        else:
            if G is None:
                G = pg.BDLTree(d, torch.int32, leaf=LEAF, X=1 << 14, device=dev, split=split) \
                    if kind == "bdl" else pg.B1Tree(d, torch.int32, leaf=LEAF, device=dev, split=split)
            t, _ = wall_ms(torch, lambda: G.insert(c))
        ms.append(t)
    return G, ms


def warm_dynamic(torch, pg, datagen, d, dev):
    """First launches of the dynamic trees' kernels (insert, erase, k-NN for
    each kind and split rule at dimension d), so that timed calls do not
    include loading them."""
    x = torch.from_numpy(datagen.uniform_int(60_000, d, seed=99)).to(dev)
    for split in ("object", "spatial"):
        for kind in ("bdl", "b1", "b2"):
            G, _ = grow_tree(torch, pg, kind, d, [x[:40_000], x[40_000:]], dev, split)
            G.erase(x[:10_000])
            for k in (2, 5, 10):
                G.knn(x[:5_000], k)
            del G
    torch.cuda.synchronize()


def form_sec63(torch, pg, datagen, dev, n=N):
    """The BDL-tree against its two baselines under the protocols of
    Section 6.3 (Figure 3: the 7-D uniform 10M set -- construction in one
    batch, 10 batches of 10% inserted into an empty tree, 10 batches of 10%
    erased from the full tree, k-NN of every point for k = 5 -- each with
    object- and spatial-median splits) and of the
    appendix on incrementally built trees (each tree grown from 20 batches of
    5% of the 2-D VisualVar-style and the 7-D uniform 10M sets, then k-NN of
    every point for k = 2..11).  Throughputs are operations per second."""
    import numpy as np
    kinds = ("bdl", "b1", "b2")
    out = {"n": n, "workload": "Section 6.3 protocols: 7-D uniform int32 10M (construction, 10x10% insert, "
                       "10x10% erase, k-NN k=5 of all points; object and spatial median); grown from 20x5% batches, k-NN of all "
                       "points for k=2..11 on 2-D VisualVar-style and 7-D uniform 10M; leaf 16, X=2^14"}
    warm_dynamic(torch, pg, datagen, 7, dev)
    warm_dynamic(torch, pg, datagen, 2, dev)
    x7 = torch.from_numpy(datagen.uniform_int(n, 7, seed=63)).to(dev)
    tenth = list(torch.chunk(x7, 10))
    order = torch.from_numpy(datagen.rng(64).permutation(n)).to(dev)
    erase_batches = [x7.index_select(0, b) for b in torch.chunk(order, 10)]
    fig3 = {}
    for split, kind in [(sp, kd) for sp in ("object", "spatial") for kd in kinds]:
        log(f"sec63 7d {split} {kind}: construction + k-NN k=5")
        G, ms = grow_tree(torch, pg, kind, 7, [x7], dev, split)
        build = ms[0]
        G.knn(x7[:4096], 5)
        knn5 = timed(torch, lambda: G.knn(x7, 5), reps=1)
        log(f"sec63 7d {split} {kind}: 10 erases of 10%")
        era = []
        for E in erase_batches:
            t, cnt = wall_ms(torch, lambda: G.erase(E))
            era.append(t)
        left = G.size()
        del G
        log(f"sec63 7d {split} {kind}: 10 inserts of 10%")
        G, ins = grow_tree(torch, pg, kind, 7, tenth, dev, split)
        del G
        torch.cuda.empty_cache()
        fig3[f"{split}_{kind}"] = {"construction_ms": build, "construction_pts_s": n / (build * 1e-3),
                      "insert_ms_total": float(np.sum(ins)), "insert_pts_s": n / (np.sum(ins) * 1e-3),
                      "erase_ms_total": float(np.sum(era)), "erase_pts_s": n / (np.sum(era) * 1e-3),
                      "knn5_ms": knn5, "knn5_qps": n / (knn5 * 1e-3),
                      "insert_ms_per_batch": [round(v, 2) for v in ins],
                      "erase_ms_per_batch": [round(v, 2) for v in era], "live_after_erase": left}
    out["fig3_7d_uniform"] = fig3
    del tenth, erase_batches, order
    vary = {}
    for name, pts in (("2d_visualvar", None), ("7d_uniform", x7)):
        if pts is None:
            pts = torch.from_numpy(datagen.visual_var(n, 2, seed=65)).to(dev)
        d = pts.shape[1]
        chunks = list(torch.chunk(pts, 20))
        res = {}
        for kind in kinds:
            log(f"sec63 {name} {kind}: grow from 20 batches of 5%, k-NN k=2..11")
            G, ms = grow_tree(torch, pg, kind, d, chunks, dev)
            qps = {}
            for k in range(2, 12):
                G.knn(pts[:4096], k)  # first launch of this k's kernels
                qps[str(k)] = n / (timed(torch, lambda: G.knn(pts, k), reps=1) * 1e-3)
            res[kind] = {"grow_ms_total": float(np.sum(ms)), "knn_qps": qps}
            if kind == "b2":
                res[kind]["levels"] = G.stats()[1]
            del G
            torch.cuda.empty_cache()
        vary[name] = res
        del chunks
    out["vary_k_grown_20x5pct"] = vary
    return out


def form_ksweep(torch, pg, datagen, dev, n=2_000_000):
    """The appendix's k sweep on incrementally built trees, at a size that
    fits the default run: the 2-D VisualVar-style set (n = 2M, seed 65)
    grown into each dynamic tree from 20 batches of 5%, then k-NN of all
    points for k = 2, 5, 11."""
    import numpy as np
    warm_dynamic(torch, pg, datagen, 2, dev)
    pts = torch.from_numpy(datagen.visual_var(n, 2, seed=65)).to(dev)
    chunks = list(torch.chunk(pts, 20))
    out = {"workload": f"2-D VisualVar-style n={n} int32, grown from 20 x 5% batches, all-points k-NN"}
    ks = (2, 5, 11)
    for kind in ("bdl", "b1", "b2"):
        G, ms = grow_tree(torch, pg, kind, 2, chunks, dev)
        res = {"grow_ms_total": float(np.sum(ms))}
        for k in ks:
            G.knn(pts, k)  # first launch of this k's kernels, and the handle's scratch at full size
            t = timed(torch, lambda: G.knn(pts, k), reps=1)
            res[f"k{k}_ms"] = t
            res[f"k{k}_qps"] = n / (t * 1e-3)
        # a lower bound of the bytes: each query read, its k (id, distance) written
        res["roofline"] = roof(n * (8 + 11 * 16), res["k11_ms"], "bdl_knn_kernel (k = 11)",
                               "lower bound: query coordinates read + k int64 ids and int64 distances written "
                               "(visits unmodelled on this set)")
        if kind == "b2":
            res["levels"] = G.stats()[1]
        out[kind] = res
        del G
        torch.cuda.empty_cache()
    return out


def form_table1(torch, pg, datagen, dev, n=N):
    """The kd-tree rows of Table 1 on their own shapes (10M uniform int32
    points): build in 2-D and 5-D, all-points k-NN in 2-D (k = 10; the
    paper does not state its k), range search in 2-D (a square of half side
    512 around every point), the k-NN graph in 2-D (k = 10), and the
    batch-dynamic tree in 5-D (construction over all points; ten 10%
    batches inserted into an empty tree, then ten 10% batches erased, both
    totals, as in Section 6.3)."""
    import numpy as np
    out = {"workload": f"Table 1 kd-tree rows: {n:,} uniform int32 points in [0,2^20)^d, leaf 16"}
    holder = {}
    x2 = torch.from_numpy(datagen.uniform_int(n, 2, seed=11)).to(dev)
    x5 = torch.from_numpy(datagen.uniform_int(n, 5, seed=12)).to(dev)
    out["build_2d_ms"] = timed(torch, lambda: holder.__setitem__("t", pg.kdtree_build(x2, leaf=LEAF)))
    t2 = holder.pop("t")
    out["build_5d_ms"] = timed(torch, lambda: holder.__setitem__("t", pg.kdtree_build(x5, leaf=LEAF)))
    holder.pop("t")
    idx = torch.empty((n, K), dtype=torch.int32, device=dev)
    dist = torch.empty((n, K), dtype=torch.int64, device=dev)
    out["knn_2d_ms"] = timed(torch, lambda: t2.knn_all(K, out=(idx, dist)))
    out["knn_graph_2d_ms"] = timed(torch, lambda: t2.knn_graph(K, out=(idx, dist)))
    del idx, dist
    boxes = torch.from_numpy(datagen.range_boxes(x2.cpu().numpy(), 512)).to(dev)
    t2.range_search(boxes)  # first launch of the range kernels
    out["range_2d_ms"] = timed(torch, lambda: t2.range_search(boxes))
    del t2, boxes
    torch.cuda.empty_cache()
    warm_dynamic(torch, pg, datagen, 5, dev)
    G, ms = grow_tree(torch, pg, "bdl", 5, [x5], dev)
    out["bdl_construction_5d_ms"] = ms[0]
    del G
    tenth = list(torch.chunk(x5, 10))
    G, ins = grow_tree(torch, pg, "bdl", 5, tenth, dev)
    out["bdl_insert_5d_ms_total"] = float(np.sum(ins))
    era = []
    for E in tenth:
        t, _ = wall_ms(torch, lambda: G.erase(E))
        era.append(t)
    out["bdl_delete_5d_ms_total"] = float(np.sum(era))
    out["bdl_live_after_delete"] = G.size()
    del G, tenth, x2, x5
    torch.cuda.empty_cache()
    return out


def form_wspd(torch, pg, datagen, dev):
    """The WSPD row of Table 1: 10M uniform 2-D int32 points (seed 11), the
    object-median tree with leaf size 1, separation s = 2: the build and the
    decomposition (pairs of heap nodes)."""
    pts = datagen.uniform_int(N, 2, seed=11)
    x = torch.from_numpy(pts).to(dev)
    holder = {}
    build_ms = timed(torch, lambda: holder.__setitem__("t", pg.kdtree_build(x, leaf=1)))
    t = holder["t"]
    pairs = t.wspd(2.0)
    P = pairs.shape[0]
    buf = torch.empty((P, 2), dtype=torch.int32, device=dev)
    wspd_ms = timed(torch, lambda: t.wspd(2.0, out=buf))
    return {"workload": "WSPD, 2-D n=10M int32 uniform, leaf 1, s=2", "build_ms": build_ms,
            "wspd_ms": wspd_ms, "pairs": P, "pairs_per_point": P / N,
            "pairs_per_s": P / (wspd_ms * 1e-3),
            "roofline": roof(P * (8 + 2 * 2 * 2 * 4), wspd_ms, "wspd rounds (test + scatter + scans)",
                             "per output pair: its 8 bytes and the two node boxes tested")}


def form_small_2d(torch, pg, datagen, dev, with_oracle):
    """The small correctness workload (10,000 uniform 2-D int32 points, all
    queried, k = 10, leaf 16): GPU build and k-NN (launch-bound at this
    size), and the oracle's brute force and kd-tree search on one core."""
    n = 10_000
    pts = datagen.uniform_int(n, 2, seed=1)
    x = torch.from_numpy(pts).to(dev)
    holder = {}
    out = {"workload": "2-D n=10,000 int32 uniform, k=10, leaf 16, all points"}
    out["build_ms"] = timed(torch, lambda: holder.__setitem__("t", pg.kdtree_build(x, leaf=LEAF)))
    t = holder["t"]
    out["knn_ms"] = timed(torch, lambda: t.knn_all(K))
    if with_oracle:
        import oracle
        t0 = time.perf_counter()
        oracle.knn_brute(pts, pts, K)
        out["oracle_brute_s"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        T = oracle.KdTree(pts, leaf=LEAF)
        T.knn(pts, K)
        out["oracle_kdtree_s"] = time.perf_counter() - t0
        out["oracle_cores"] = 1
    return out


def form_batch(torch, pg, datagen, dev, loop_clouds):
    """4,096 sphere clouds (sizes log-uniform in [256, 65536]), per-cloud
    all-points k = 16 in one persistent launch, against the per-cloud static
    method; plus the k-NN backward over the same clouds (leaf-order batched
    kernel, and the generic one)."""
    import numpy as np
    sizes = datagen.cloud_sizes(4096, seed=4)
    pts, offs = datagen.sphere_clouds(sizes, seed=44)
    Ntot = len(pts)
    x = torch.from_numpy(pts).to(dev)
    tune = pg.batch_autotune(x, offs, 16)
    Bk = pg.BatchKnn(offs, 3, device=dev, **tune)
    idx = torch.empty((Ntot, 16), dtype=torch.int32, device=dev)
    d2 = torch.empty((Ntot, 16), dtype=torch.float32, device=dev)
    batch_ms = timed(torch, lambda: Bk.knn_self(x, 16, out=(idx, d2)))
    # per-cloud static method on the first loop_clouds clouds (projected)
    nc = min(loop_clouds, 4096)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(nc):
        t = pg.kdtree_build(x[int(offs[c]):int(offs[c + 1])], leaf=16)
        t.knn_all(16)
    torch.cuda.synchronize()
    loop_s = (time.perf_counter() - t0) * 4096 / nc
    g = torch.randn((Ntot, 16), dtype=torch.float32, device=dev)
    grad = torch.empty_like(x)
    # the leaf-order backward of the batched launch (its trees are the last
    # knn_self's), and the generic reverse-CSR backward for comparison
    bwd_ms = timed(torch, lambda: Bk.backward(x, idx, d2, g, out=grad))
    gen_ms = timed(torch, lambda: pg.knn_backward(x, x, idx, g, grad_q=grad, self_mode=True))
    fast_ms = timed(torch, lambda: pg.knn_backward(x, x, idx, g, grad_q=grad, self_mode=True,
                                                   deterministic=False))
    vi, vp = VISITS["sphere_clouds_all_points"]
    fwd_b = sum(build_bytes(int(n), 3, tree_levels(int(n))) for n in sizes) + \
        Ntot * knn_bytes(3, 16, 4, 4, vi, vp)
    bwd_b = Ntot * 16 * 8 + Ntot * 12 * 2  # idx + g per pair; points read, gradient written
    return {"workload": "4,096 unit-sphere clouds (+N(0,0.01^2)), sizes log-uniform [256,65536], "
                        f"{Ntot} points, per-cloud all-points k=16, float32",
            "roofline": roof(fwd_b, batch_ms, "batch_kernel (builds + searches, one launch)",
                             f"per-cloud builds (build_bytes) + searches ({vi} internal nodes, "
                             f"{vp} points per query, oracle on 256 clouds)"),
            "backward_roofline": roof(bwd_b, bwd_ms, "bwd_* (leaf-order batched backward)",
                                      "8 B per (query, neighbour) pair (index, gradient) + the "
                                      "points read and the gradient written"),
            "tune": tune, "batched_ms": batch_ms, "clouds_per_s": 4096 / (batch_ms * 1e-3),
            "points_per_s": Ntot / (batch_ms * 1e-3),
            "per_cloud_loop_ms": loop_s * 1e3, "per_cloud_loop_sample_clouds": nc,
            "speedup_vs_per_cloud_loop": loop_s * 1e3 / batch_ms,
            "backward_ms": bwd_ms, "backward_pairs_per_s": Ntot * 16 / (bwd_ms * 1e-3),
            "backward_generic_ms": gen_ms, "backward_atomic_ms": fast_ms}


# Oracle visit counts per box on the range workload (100,000 sampled boxes):
# node boxes tested 52.222, points tested 33.489, results 10.552.
R_NODES, R_PTS = 52.222, 33.489


def range_bytes_per_query(d, results, report):
    """Algorithmic bytes of one range query: the box (8d), node boxes tested
    (8d each), points tested (4(d+1) each), and the output: the count (4) in
    the counting pass, the offset (8) and 4 bytes per result in the
    reporting pass."""
    tree = 8 * d + 8 * d * R_NODES + 4 * (d + 1) * R_PTS
    return tree + (8 + 4 * results if report else 4)


def form_range(torch, pg, datagen, dev, with_oracle):
    """Orthogonal range search, the 2-D row of the paper's Table 1 read as:
    10M uniform int32 points in [0,2^20)^2 and one closed square of half side
    512 around every point (about 10.6 points per square).  ``search_ms``
    times pg_range_search (boxes checked and ordered once, counting pass,
    prefix sum, reporting pass); ``count_ms`` / ``report_ms`` time the two
    separate calls (each orders the boxes itself)."""
    import numpy as np
    pts = datagen.uniform_int(N, 2, seed=2)
    boxes = datagen.range_boxes(pts, 512)
    x = torch.from_numpy(pts).to(dev)
    b = torch.from_numpy(boxes).to(dev)
    holder = {}
    build_ms = timed(torch, lambda: holder.__setitem__("t", pg.kdtree_build(x, leaf=LEAF)))
    t = holder["t"]
    counts, off, total = t.range_count(b, offsets=True)
    rows = torch.empty(total, dtype=torch.int32, device=dev)
    count_ms = timed(torch, lambda: t.range_count(b, offsets=True))
    report_ms = timed(torch, lambda: t.range_report(b, off, rows))
    search_ms = timed(torch, lambda: t.range_search(b, capacity=total))
    out = {"workload": "2-D n=10M int32 uniform, a closed square of half side 512 around "
                       "every point, leaf 16",
           "build_ms": build_ms, "search_ms": search_ms, "count_ms": count_ms,
           "report_ms": report_ms, "results_per_query": total / N,
           "qps": N / (search_ms * 1e-3)}
    res = total / N
    for name, ms, rep in (("count", count_ms, False), ("report", report_ms, True)):
        gbs = range_bytes_per_query(2, res, rep) * N / (ms * 1e-3) / 1e9
        out[f"{name}_algorithmic_gbs"] = gbs
        out[f"{name}_roofline_frac"] = gbs / HBM_PEAK_GBS
    out["roofline"] = roof((range_bytes_per_query(2, res, False) + range_bytes_per_query(2, res, True))
                           * N, search_ms, "range_kernel (counting and reporting walks)",
                           f"per box: the box, {R_NODES} node boxes and {R_PTS} points tested "
                           "(oracle), count, offset and rows; both passes")
    if with_oracle:
        import oracle
        sample = 100_000
        T = oracle.KdTree(pts, leaf=LEAF)
        t0 = time.perf_counter()
        T.range(boxes[:sample])
        out["oracle_qps_1core"] = sample / (time.perf_counter() - t0)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", choices=["int", "float"], default="int")
    ap.add_argument("--cpu-sample", type=int, default=100_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="all",
                    help="other forms to measure after the headline step: all, none, or a "
                         "comma list of static_float,clustered,spatial,bdl,baselines,ksweep,batch,range,"
                         "graph,wspd,table1,small_2d "
                         "(sec63, the Section 6.3 protocols on 10M-point sets, runs only when named)")
    ap.add_argument("--bdl-rounds", type=int, default=10)
    ap.add_argument("--sec63-n", type=int, default=N, help="set size of the sec63 form")
    ap.add_argument("--loop-clouds", type=int, default=512,
                    help="clouds timed for the per-cloud comparison (projected to 4,096)")
    ap.add_argument("--copy-probe-mib", type=int, default=1024,
                    help="size of the device copy that measures achievable HBM bandwidth (0: skip)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the k-NN traffic summary from two rocprofv3 --pmc counter "
                         "CSVs (FETCH_SIZE, WRITE_SIZE) of a run of this script, then exit")
    ap.add_argument("--traffic-command", default="",
                    help="the profiling command recorded with --write-traffic")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic[0], args.write_traffic[1], args.dtype,
                      args.copy_probe_mib, args.traffic_command)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2207_01834_amd import _binding as pg
    from paper_2207_01834_amd import datagen

    dev = torch.device("cuda:0")
    pts = datagen.uniform_int(N, D, seed=2)
    if args.dtype == "float":
        pts = datagen.int_to_unit_float(pts)
    x = torch.from_numpy(pts).to(dev)
    dist_dtype = torch.int64 if args.dtype == "int" else torch.float32
    idx = torch.empty((N, K), dtype=torch.int32, device=dev)
    dist = torch.empty((N, K), dtype=dist_dtype, device=dev)
    torch.cuda.synchronize()

    def step(evs=None):
        if evs:
            evs[0].record()
        t = pg.kdtree_build(x, leaf=LEAF)
        if evs:
            evs[1].record()
        t.knn_all(K, out=(idx, dist))
        if evs:
            evs[2].record()
        return t

    for w in range(args.warmup):
        log(f"warmup {w + 1}/{args.warmup}")
        t = step()
        del t
    torch.cuda.synchronize()

    copy_gbs = copy_probe(torch, dev, args.copy_probe_mib)

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        t = step(evs[s])
        del t
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    build_ms = float(np.median([e[0].elapsed_time(e[1]) for e in evs]))
    knn_ms = float(np.median([e[1].elapsed_time(e[2]) for e in evs]))
    ms_per_step = wall * 1000.0 / args.steps
    log(f"step {ms_per_step:.3f} ms (build {build_ms:.3f} ms, knn {knn_ms:.3f} ms)")

    dbytes = 8 if args.dtype == "int" else 4
    launch_bytes = bytes_per_query(dbytes) * N
    achieved = launch_bytes / (knn_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.dtype)
    line = {
        "metric": "kNN queries/sec + build Mpts/s (3D n=10M k=10), % HBM roofline, vs CPU oracle",
        "value": N / (ms_per_step * 1e-3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64" if args.dtype == "int" else "f32",
        "data": "synthetic",
        "config": {
            "workload": ("static 3-D kd-tree build + all-points k-NN: n=10,000,000 points, "
                         + ("int32 coordinates uniform in [0,2^20)^3, exact int64 squared distances"
                            if args.dtype == "int" else
                            "float32 coordinates uniform in [0,1)^3 (int grid / 2^20), float32 distances")
                         + ", k=10, leaf size 16, queries = all points"),
            "n": N, "d": D, "k": K, "leaf": LEAF, "seed": 2,
        },
        "build_mpts_s": N / (build_ms * 1e-3) / 1e6,
        "knn_qps": N / (knn_ms * 1e-3),
        "build_ms": build_ms,
        "hbm_copy_gbs": copy_gbs,
        "knn_ms": knn_ms,
        "roofline": {
            "bound": "hbm",
            "kernel": "knn_static_kernel (all-points)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": launch_bytes,
            "algorithmic_bytes_per_query": bytes_per_query(dbytes),
        },
        "build_roofline": roof(build_bytes(N, D, tree_levels(N)), build_ms, "build (all kernels)",
                               "n(8d+4) + L n (8d+12): ingest, then per level one key read and "
                               "one record read and write"),
    }
    del idx, dist, x
    torch.cuda.empty_cache()
    forms = ["static_float", "clustered", "spatial", "bdl", "baselines", "ksweep", "batch", "range", "graph",
             "wspd", "table1", "small_2d"] \
        if args.forms == "all" else \
        [f for f in args.forms.split(",") if f and f != "none"]
    out = {}
    for f in forms:
        log(f"form {f}")
        if f == "static_float":
            out[f] = form_static_float(torch, pg, datagen, dev)
        elif f == "clustered":
            out[f] = form_clustered(torch, pg, datagen, dev)
        elif f == "bdl":
            out[f] = form_bdl(torch, pg, datagen, dev, args.bdl_rounds, not args.no_cpu_baseline)
        elif f == "batch":
            out[f] = form_batch(torch, pg, datagen, dev, args.loop_clouds)
        elif f == "spatial":
            out[f] = form_spatial(torch, pg, datagen, dev)
        elif f == "baselines":
            out[f] = form_baselines(torch, pg, datagen, dev, args.bdl_rounds)
        elif f == "graph":
            out[f] = form_graph(torch, pg, datagen, dev)
        elif f == "small_2d":
            out[f] = form_small_2d(torch, pg, datagen, dev, not args.no_cpu_baseline)
        elif f == "table1":
            out[f] = form_table1(torch, pg, datagen, dev)
        elif f == "sec63":
            out[f] = form_sec63(torch, pg, datagen, dev, args.sec63_n)
        elif f == "range":
            out[f] = form_range(torch, pg, datagen, dev, not args.no_cpu_baseline)
        elif f == "wspd":
            out[f] = form_wspd(torch, pg, datagen, dev)
        elif f == "ksweep":
            out[f] = form_ksweep(torch, pg, datagen, dev)
        else:
            raise SystemExit(f"unknown form {f}")
        torch.cuda.empty_cache()
    if out:
        line["forms"] = out
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pts, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
