"""The seeded input generators: same arguments, same bytes; coordinate
ranges as stated; the VisualVar-style set's density varies across clusters
and its rows carry no walk order."""
import numpy as np

from paper_2207_01834_amd import datagen


def test_generators_are_deterministic():
    a = datagen.uniform_int(5_000, 3, seed=4)
    assert np.array_equal(a, datagen.uniform_int(5_000, 3, seed=4))
    assert not np.array_equal(a, datagen.uniform_int(5_000, 3, seed=5))
    assert np.array_equal(datagen.visual_var(5_000, 2, seed=6), datagen.visual_var(5_000, 2, seed=6))
    c1, q1 = datagen.clustered(3_000, 5, seed=3, n_queries=500, query_seed=33)
    c2, q2 = datagen.clustered(3_000, 5, seed=3, n_queries=500, query_seed=33)
    assert np.array_equal(c1, c2) and np.array_equal(q1, q2)
    s = datagen.cloud_sizes(64, seed=4)
    p1, o1 = datagen.sphere_clouds(s, seed=44)
    p2, o2 = datagen.sphere_clouds(s, seed=44)
    assert np.array_equal(p1, p2) and np.array_equal(o1, o2)


def test_ranges_and_types():
    u = datagen.uniform_int(20_000, 4, seed=1)
    assert u.dtype == np.int32 and u.min() >= 0 and u.max() < (1 << 20)
    f = datagen.int_to_unit_float(u)
    assert f.dtype == np.float32 and np.array_equal((f.astype(np.float64) * (1 << 20)).astype(np.int64), u)
    v = datagen.visual_var(20_000, 3, seed=2)
    assert v.dtype == np.int32 and v.shape == (20_000, 3) and v.min() >= 0 and v.max() < (1 << 20)
    s = datagen.cloud_sizes(500, seed=7)
    assert s.min() >= 256 and s.max() <= 65536
    _, off = datagen.sphere_clouds(s[:10], seed=8)
    assert off[0] == 0 and np.array_equal(np.diff(off), s[:10])


def test_visual_var_density_varies_and_rows_are_shuffled():
    from scipy.spatial import cKDTree
    n = 400_000
    v = datagen.visual_var(n, 2, seed=3).astype(np.float64)
    u = datagen.uniform_int(n, 2, seed=3).astype(np.float64)

    def spread(p):
        d, _ = cKDTree(p).query(p[::200], k=2)
        lo, hi = np.percentile(d[:, 1], [5, 95])
        return hi / max(lo, 1.0)
    # nearest-neighbour distances spread far wider than on uniform points
    assert spread(v) > 5 * spread(u)
    # consecutive rows are not neighbours along a walk: a row's successor is
    # about as far as a random point
    step = np.linalg.norm(v[1:] - v[:-1], axis=1).mean()
    rand = np.linalg.norm(v[1:] - v[np.random.default_rng(0).permutation(n - 1)], axis=1).mean()
    assert step > 0.8 * rand
