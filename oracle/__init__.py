"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct CPU implementations of what the GPU library
computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package; the GPU library never calls it
and shares no code with it.

Parts (each function cites the passage it follows):
  * ``knn_brute``  -- the k-NN definition written out (C, ``or_knn_brute``);
  * ``KdTree``     -- the static kd-tree with object-median splits and its
                      k-NN search (C, ``or_kd_build`` / ``or_kd_knn``);
  * ``bdl_model``  -- the BDL-tree's logarithmic method on point sets
                      (Algorithms 3 and 4), in Python;
  * ``grad``       -- the closed-form FP64 gradient of summed k-NN squared
                      distances and central finite differences, in NumPy;
  * ``KdTree.wspd`` -- the well-separated pair decomposition from the
                      kd-tree (C, ``or_wspd``);
  * ``spatial_tree`` -- the kd-tree by spatial-median splits, split until
                      a node holds at most ``leaf`` points (C,
                      ``or_sp_build``);
  * ``knn_graph_brute`` -- the k-NN graph (each point's k nearest other
                      points) from the k-NN definition;
  * ``range_brute`` / ``KdTree.range`` -- the orthogonal range query written
                      out, and on the tree (C, ``or_range_brute`` /
                      ``or_kd_range``).

Readings of the paper adopted where it is silent (also listed in the design
notes): ties in distance go to the smaller id; squared distances are exact
int64 for int32 coordinates and FP64 for float32 coordinates; split
dimension = level mod d; split rank floor((2j+1)n/2^(l+1)) under
(coordinate, index); leaves at depth L = min{L : ceil(n/2^L) <= leaf}.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

DT_INT, DT_F32 = 0, 1


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            from . import build_oracle
            build_oracle.build()
        L = ctypes.CDLL(_SO)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.or_knn_brute.argtypes = [vp, vp, vp, i64, i32, i32, vp, i64, i32, vp, vp, i32]
        L.or_knn_brute.restype = i32
        L.or_kd_build.argtypes = [vp, i64, i32, i32, i32]
        L.or_kd_build.restype = vp
        L.or_kd_free.argtypes = [vp]
        L.or_kd_free.restype = None
        L.or_kd_levels.argtypes = [vp]
        L.or_kd_levels.restype = i32
        L.or_kd_export.argtypes = [vp, vp, vp]
        L.or_kd_export.restype = None
        L.or_kd_knn.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp, vp]
        L.or_kd_knn.restype = i32
        L.or_sp_build.argtypes = [vp, i64, i32, i32, i32, i32]
        L.or_sp_build.restype = vp
        L.or_sp_free.argtypes = [vp]
        L.or_sp_free.restype = None
        L.or_sp_nodes.argtypes = [vp]
        L.or_sp_nodes.restype = i64
        L.or_sp_depth.argtypes = [vp]
        L.or_sp_depth.restype = i32
        L.or_sp_export.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.or_sp_export.restype = None
        L.or_wspd.argtypes = [vp, ctypes.c_double, vp, i64]
        L.or_wspd.restype = i64
        L.or_range_brute.argtypes = [vp, vp, vp, i64, i32, i32, vp, i64, vp, vp, vp]
        L.or_range_brute.restype = i32
        L.or_kd_range.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp]
        L.or_kd_range.restype = i32
        _lib = L
    return _lib


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.int32:
        return DT_INT
    if a.dtype == np.float32:
        return DT_F32
    raise TypeError(f"oracle takes int32 or float32 coordinates, got {a.dtype}")


def _ptr(a):
    return None if a is None else a.ctypes.data


def _outputs(m, k, dt):
    ids = np.empty((m, k), dtype=np.int64)
    dist = np.empty((m, k), dtype=np.int64 if dt == DT_INT else np.float64)
    return ids, dist


def knn_brute(points, queries, k, ids=None, alive=None, nthreads=1):
    """The definition: for every query the k smallest (D, id) keys, ascending.
    Returns (ids int64 [m][k], dist int64 or float64 [m][k]); missing slots
    hold id -1 and distance INT64_MAX / +inf."""
    points = np.ascontiguousarray(points)
    queries = np.ascontiguousarray(queries, dtype=points.dtype)
    dt = _dtype_code(points)
    n, d = points.shape
    m = queries.shape[0]
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
    if alive is not None:
        alive = np.ascontiguousarray(alive, dtype=np.uint8)
    out_id, out_d = _outputs(m, k, dt)
    rc = lib().or_knn_brute(_ptr(points), _ptr(ids), _ptr(alive), n, d, dt,
                            _ptr(queries), m, k, _ptr(out_id), _ptr(out_d), int(nthreads))
    if rc != 0:
        raise ValueError("or_knn_brute: bad arguments")
    return out_id, out_d


def knn_graph_brute(points, k, nthreads=1):
    """The k-NN graph (Section 2, third module: graphs generated from the
    kd-tree's k-NN search), written out: row i holds the k smallest
    (D(p_i, p_j), j) keys over the points j != i, ascending; missing slots
    hold id -1 and distance INT64_MAX / +inf.  Built from the definition's
    k+1 nearest of every point with row i's own entry removed (when more
    than k identical points precede it, its own entry is not among them and
    the first k are kept)."""
    points = np.ascontiguousarray(points)
    n = points.shape[0]
    ids, dist = knn_brute(points, points, k + 1, nthreads=nthreads)
    own = ids == np.arange(n, dtype=np.int64)[:, None]
    keep = ~own
    keep[own.sum(axis=1) == 0, k] = False  # self not listed: drop the (k+1)-th
    out_i = ids[keep].reshape(n, k)
    out_d = dist[keep].reshape(n, k)
    return out_i, out_d


def _offsets(counts):
    off = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def range_brute(points, boxes, ids=None, alive=None):
    """The orthogonal range query written out (reading: a query is a closed
    box [lo, hi], boxes [m][2][d] = lo then hi; the result is every live
    point inside it).  Returns (counts int64 [m], offsets int64 [m+1],
    ids int64 [total]) with each box's ids in row order."""
    points = np.ascontiguousarray(points)
    dt = _dtype_code(points)
    n, d = points.shape
    boxes = np.ascontiguousarray(boxes, dtype=points.dtype).reshape(-1, 2, d)
    m = boxes.shape[0]
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
    if alive is not None:
        alive = np.ascontiguousarray(alive, dtype=np.uint8)
    counts = np.zeros(m, dtype=np.int64)
    rc = lib().or_range_brute(_ptr(points), _ptr(ids), _ptr(alive), n, d, dt, _ptr(boxes), m,
                              _ptr(counts), None, None)
    if rc != 0:
        raise ValueError("or_range_brute: bad arguments")
    off = _offsets(counts)
    out = np.empty(int(off[-1]), dtype=np.int64)
    lib().or_range_brute(_ptr(points), _ptr(ids), _ptr(alive), n, d, dt, _ptr(boxes), m,
                         _ptr(counts), _ptr(off), _ptr(out))
    return counts, off, out


class KdTree:
    """Static kd-tree by object-median splits (Appendix C, Algorithm 1 and the
    proof of its work bound: one median partition per level), read as: split
    dimension = level mod d, split position floor((2j+1)n/2^(l+1)) under the
    key (coordinate, row index), all leaves at depth L."""

    def __init__(self, points, leaf=16):
        self.points = np.ascontiguousarray(points)
        self.dt = _dtype_code(self.points)
        self.n, self.d = self.points.shape
        self.leaf = leaf
        self._h = lib().or_kd_build(_ptr(self.points), self.n, self.d, self.dt, leaf)
        if not self._h:
            raise ValueError("or_kd_build: bad arguments")
        self.levels = lib().or_kd_levels(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_kd_free(h)
            self._h = None

    def export(self):
        """(split values of heap nodes 1..2^L-1 as float64, rows in leaf order)."""
        ni = (1 << self.levels) - 1
        splits = np.empty(ni, dtype=np.float64)
        perm = np.empty(self.n, dtype=np.int64)
        lib().or_kd_export(self._h, _ptr(splits), _ptr(perm))
        return splits, perm

    def leaf_ranges(self):
        L = self.levels
        j = np.arange((1 << L) + 1, dtype=object)
        return np.array([(int(x) * self.n) >> L for x in j], dtype=np.int64)

    def knn(self, queries, k, ids=None, alive=None, nthreads=1):
        """Appendix C single-query search for every query; returns
        (ids, dist, counters) with counters = [internal nodes visited,
        leaves added, points whose distance was computed] summed.  With
        nthreads > 1 the queries are searched in that many static chunks on
        as many threads (each search is the same serial search; the C call
        releases the interpreter lock), which changes no result."""
        queries = np.ascontiguousarray(queries, dtype=self.points.dtype)
        m = queries.shape[0]
        if ids is not None:
            ids = np.ascontiguousarray(ids, dtype=np.int64)
        if alive is not None:
            alive = np.ascontiguousarray(alive, dtype=np.uint8)
        out_id, out_d = _outputs(m, k, self.dt)
        nthreads = max(1, min(int(nthreads), m))
        bounds = [m * t // nthreads for t in range(nthreads + 1)]
        counters = np.zeros((nthreads, 3), dtype=np.int64)

        def run(t):
            a, b = bounds[t], bounds[t + 1]
            return lib().or_kd_knn(self._h, _ptr(ids), _ptr(alive), _ptr(queries[a:b]), b - a, k,
                                   _ptr(out_id[a:b]), _ptr(out_d[a:b]), _ptr(counters[t]))
        if nthreads == 1:
            rcs = [run(0)]
        else:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(nthreads) as ex:
                rcs = list(ex.map(run, range(nthreads)))
        if any(rc != 0 for rc in rcs):
            raise ValueError("or_kd_knn: bad arguments")
        return out_id, out_d, counters.sum(axis=0)

    def wspd(self, s=2.0):
        """The well-separated pair decomposition generated from this tree
        (leaf size 1): int64 [P][2] heap node pairs (a from the first
        child's side of the internal node that started the pairing), in the
        order the recursion emits them."""
        cnt = lib().or_wspd(self._h, float(s), None, 0)
        if cnt < 0:
            raise ValueError("or_wspd: s must be positive and finite, and the leaf size 1")
        out = np.empty((cnt, 2), dtype=np.int64)
        lib().or_wspd(self._h, float(s), _ptr(out), cnt)
        return out

    def node_range(self, h):
        """Leaf-order positions [lo, hi) of heap node h."""
        l = int(h).bit_length() - 1
        j = int(h) - (1 << l)
        return (j * self.n) >> l, ((j + 1) * self.n) >> l

    def range(self, boxes, ids=None, alive=None):
        """Range search on the tree (boxes inside the query report whole,
        boxes missing it are skipped); returns (counts, offsets, ids in leaf
        order, counters = [node boxes tested, points tested])."""
        boxes = np.ascontiguousarray(boxes, dtype=self.points.dtype).reshape(-1, 2, self.d)
        m = boxes.shape[0]
        if ids is not None:
            ids = np.ascontiguousarray(ids, dtype=np.int64)
        if alive is not None:
            alive = np.ascontiguousarray(alive, dtype=np.uint8)
        counts = np.zeros(m, dtype=np.int64)
        counters = np.zeros(2, dtype=np.int64)
        rc = lib().or_kd_range(self._h, _ptr(ids), _ptr(alive), _ptr(boxes), m, _ptr(counts),
                               None, None, None)
        if rc != 0:
            raise ValueError("or_kd_range: bad arguments")
        off = _offsets(counts)
        out = np.empty(int(off[-1]), dtype=np.int64)
        lib().or_kd_range(self._h, _ptr(ids), _ptr(alive), _ptr(boxes), m, _ptr(counts),
                          _ptr(off), _ptr(out), _ptr(counters))
        return counts, off, out, counters


class SpatialTree:
    """A kd-tree by spatial-median splits, as arrays (nodes numbered
    breadth-first: the root is 0, a level's nodes in leaf order, the
    children of an internal node consecutive):
      split  float64 [N]  cut value (0 for leaves)
      dim    int32   [N]  cut dimension (-1 for leaves)
      child  int64   [N]  first child (-1 for leaves); the second is child+1
      lo, hi int64   [N]  the node's leaf-order positions [lo, hi)
      level  int32   [N]  depth of the node (root 0)
      perm   int64   [n]  input rows in leaf order
      depth  int          levels (1 + the deepest node's depth)"""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    @property
    def leaves(self):
        return np.nonzero(self.child < 0)[0]

    def leaf_sizes(self):
        lv = self.leaves
        return self.hi[lv] - self.lo[lv]


def spatial_tree(points, leaf=16, rule="cycle", space="cell"):
    """Spatial-median kd-tree (Section 6.3: the node's space cut in half along
    a dimension; Section 5: split until a node holds a small constant number
    of points), read as: a node holding at most ``leaf`` points, or only
    identical points, is a leaf; the root's space is the points' bounding
    box; a node cuts its cell (space "cell") or the bounding box of its own
    points (space "points") along dimension depth mod d (rule "cycle") or
    the space's widest side, lowest dimension on ties (rule "widest"); the
    cut of [lo, hi] is floor((lo + hi + 1) / 2) for int32, the float nearest
    (lo + hi) / 2 for float32 (the next float above lo when that is lo
    itself), lo when lo == hi; coordinate < cut goes left (cell [lo, cut-]),
    the rest right (cell [cut, hi]), each side in the parent's order.
    Returns a :class:`SpatialTree`."""
    points = np.ascontiguousarray(points)
    dt = _dtype_code(points)
    n, d = points.shape
    r = {"cycle": 0, "widest": 1}[rule] | {"cell": 0, "points": 2}[space]
    h = lib().or_sp_build(_ptr(points), n, d, dt, leaf, r)
    if not h:
        raise ValueError("or_sp_build: bad arguments")
    try:
        N = lib().or_sp_nodes(h)
        out = dict(split=np.empty(N, np.float64), dim=np.empty(N, np.int32),
                   child=np.empty(N, np.int64), lo=np.empty(N, np.int64),
                   hi=np.empty(N, np.int64), level=np.empty(N, np.int32),
                   perm=np.empty(n, np.int64))
        lib().or_sp_export(h, *[_ptr(out[k]) for k in ("split", "dim", "child", "lo", "hi",
                                                         "level", "perm")])
        depth = lib().or_sp_depth(h)
    finally:
        lib().or_sp_free(h)
    return SpatialTree(nodes=N, depth=depth, **out)


def tree_depth(n: int, leaf: int) -> int:
    """L = min{L : ceil(n / 2^L) <= leaf}."""
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    return L
