"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers: it holds none of the method's
arithmetic (no distances, no trees, no selection), so both the CPU oracle and
the GPU path may take their inputs from it.

Every generator uses NumPy's PCG64 bit generator seeded through
``SeedSequence(seed)``, so an input is fully determined by its arguments.

Workload shapes (Section 6, "Data Sets"; Table 1):
  * uniform hypercube points (the paper's U data sets) with integer
    coordinates in [0, 2^20)^d; the float variant divides by 2^20, which is
    exact in float32;
  * a clustered, varying-density 5-D mixture standing in for the paper's
    clustered generator (which is not available here);
  * many small clouds on the unit sphere with a thin noise shell, standing in
    for the OnSphere data set (surface thickness);
  * a variable-density random-walk generator standing in for the paper's
    VisualVar (V) data sets;
  * batch updates of 10% of the data set (Section 6.3 insertion/deletion
    experiments).
"""
from __future__ import annotations

import numpy as np

COORD_BITS = 20


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def uniform_int(n: int, d: int, seed: int, bits: int = COORD_BITS) -> np.ndarray:
    """n points, int32 coordinates uniform in [0, 2^bits)^d, row-major [n][d]."""
    g = rng(seed)
    return g.integers(0, 1 << bits, size=(n, d), dtype=np.int64).astype(np.int32)


def int_to_unit_float(x: np.ndarray, bits: int = COORD_BITS) -> np.ndarray:
    """Scale integer coordinates in [0, 2^bits) to float32 in [0, 1) exactly."""
    return (x.astype(np.float64) / float(1 << bits)).astype(np.float32)


def uniform_float(n: int, d: int, seed: int) -> np.ndarray:
    g = rng(seed)
    return g.random((n, d), dtype=np.float64).astype(np.float32)


def clustered(n: int, d: int, seed: int, n_clusters: int = 1000,
              zipf_s: float = 1.1, log_sigma=(-4.0, -1.0),
              n_queries: int = 0, query_seed: int | None = None):
    """Gaussian-mixture points: centres uniform in [0,1)^d, per-cluster sigma
    log-uniform in [10^a, 10^b], cluster of each point drawn with probability
    proportional to rank^-zipf_s.  Returns float32 points (and, when
    ``n_queries`` > 0, float32 queries drawn from the same mixture with their
    own seed)."""
    g = rng(seed)
    centres = g.random((n_clusters, d))
    sigma = 10.0 ** g.uniform(log_sigma[0], log_sigma[1], size=n_clusters)
    ranks = np.arange(1, n_clusters + 1, dtype=np.float64)
    p = ranks ** (-zipf_s)
    p /= p.sum()

    def draw(gen, count):
        cl = gen.choice(n_clusters, size=count, p=p)
        z = gen.standard_normal((count, d))
        return (centres[cl] + sigma[cl, None] * z).astype(np.float32)

    pts = draw(g, n)
    if n_queries <= 0:
        return pts
    gq = rng(query_seed if query_seed is not None else seed + 31)
    return pts, draw(gq, n_queries)


def visual_var(n: int, d: int, seed: int, restart_prob: float = 1e-4,
               radius_exp=(-3.5, -1.5), step_frac: float = 0.05,
               bits: int = COORD_BITS) -> np.ndarray:
    """Variable-density clustered int32 points in [0, 2^bits)^d, standing in
    for the paper's VisualVar data sets (Section 6, "Data Sets": a random
    walk through a local region that jumps to a random location now and
    then).  A walker starts at a uniform location with a local radius
    r = 2^bits * 10^U(radius_exp); each point lies uniformly in the cube of
    half side r around the walker, which then moves step_frac * r in a
    uniformly random direction, or, with probability ``restart_prob``, jumps to a fresh
    uniform location and draws a fresh radius (so clusters differ in density
    by the spread of ``radius_exp``).  Coordinates wrap around the domain,
    and the rows come out in a random order (a data set carries no order, so
    a batch of consecutive rows samples every cluster)."""
    g = rng(seed)
    side = float(1 << bits)
    jump = g.random(n) < restart_prob
    if n:
        jump[0] = True
    seg = np.cumsum(jump) - 1
    walks = int(seg[-1]) + 1 if n else 0
    start = g.random((walks, d)) * side
    radius = side * 10.0 ** g.uniform(radius_exp[0], radius_exp[1], size=walks)
    r = radius[seg][:, None]
    step = g.standard_normal((n, d))
    nrm = np.sqrt(np.sum(step * step, axis=1, keepdims=True))
    nrm[nrm == 0] = 1.0
    step *= step_frac * r / nrm
    # walker position before point i: its walk's start plus the steps taken
    # since then (a running sum restarted at every jump)
    run = np.cumsum(step, axis=0) - step
    first = np.flatnonzero(jump)
    pos = start[seg] + run - run[first][seg]
    del run, step
    pos += (2.0 * g.random((n, d)) - 1.0) * r
    out = np.floor(np.mod(pos, side)).astype(np.int64).clip(0, (1 << bits) - 1).astype(np.int32)
    return out[g.permutation(n)]


def cloud_sizes(n_clouds: int, seed: int, lo: int = 256, hi: int = 65536) -> np.ndarray:
    """Cloud sizes floor(exp(U(ln lo, ln hi))) (log-uniform), int64."""
    g = rng(seed)
    s = np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), size=n_clouds)))
    return np.clip(s.astype(np.int64), lo, hi)


def sphere_clouds(sizes: np.ndarray, seed: int, noise_sigma: float = 0.01):
    """Concatenated float32 3-D clouds: points u/|u| (u ~ N(0, I3)) plus
    N(0, noise_sigma^2) per coordinate.  Returns (points [N][3], offsets
    [n_clouds+1] int64)."""
    g = rng(seed)
    total = int(np.sum(sizes))
    u = g.standard_normal((total, 3))
    nrm = np.sqrt(np.sum(u * u, axis=1, keepdims=True))
    nrm[nrm == 0] = 1.0
    pts = u / nrm + noise_sigma * g.standard_normal((total, 3))
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    return pts.astype(np.float32), offs


def bdl_rounds(n_init: int, n_rounds: int, batch: int, n_queries: int, d: int,
               seed: int, bits: int = COORD_BITS):
    """Batch-dynamic workload: ``n_init`` initial int32 points, then per round
    a batch of ``batch`` fresh points to insert, the number of points to erase
    and a seed for choosing them, and ``n_queries`` fresh query points.

    The erase batch is chosen by the caller from its own live set with
    ``choose_erase`` (sampling without replacement), so that the choice is a
    function of the seed and the live set only.
    """
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(n_rounds + 1)
    g0 = np.random.Generator(np.random.PCG64(children[0]))
    init = g0.integers(0, 1 << bits, size=(n_init, d), dtype=np.int64).astype(np.int32)
    rounds = []
    for r in range(1, n_rounds + 1):
        g = np.random.Generator(np.random.PCG64(children[r]))
        ins = g.integers(0, 1 << bits, size=(batch, d), dtype=np.int64).astype(np.int32)
        q = g.integers(0, 1 << bits, size=(n_queries, d), dtype=np.int64).astype(np.int32)
        erase_seed = int(g.integers(0, 2**62))
        rounds.append({"insert": ins, "queries": q, "erase_seed": erase_seed})
    return init, rounds


def choose_erase(live_points: np.ndarray, count: int, seed: int) -> np.ndarray:
    """Sample ``count`` rows of ``live_points`` without replacement."""
    g = rng(seed)
    count = min(count, len(live_points))
    sel = g.choice(len(live_points), size=count, replace=False)
    return np.ascontiguousarray(live_points[np.sort(sel)])


def range_boxes(points: np.ndarray, half, seed: int | None = None, m: int | None = None) -> np.ndarray:
    """Closed query boxes [m][2][d] (lo, hi) centred on data points.

    With ``seed`` None every point is a centre, in row order, and ``half`` is
    the fixed half side (the all-points range workload: squares of side
    2 half + 1 around each point of a uniform set).  Otherwise ``m`` centres are
    drawn from the points and each box takes a half side per axis uniform in
    [0, half] (test inputs of mixed sizes)."""
    p = np.asarray(points)
    if seed is None:
        c = p.astype(np.float64)
        h = np.full(c.shape, float(half))
    else:
        g = rng(seed)
        c = p[g.integers(0, p.shape[0], m)].astype(np.float64)
        h = g.uniform(0.0, float(half), c.shape)
    if p.dtype == np.int32:
        h = np.floor(h)
    return np.ascontiguousarray(np.stack([c - h, c + h], axis=1).astype(p.dtype))
