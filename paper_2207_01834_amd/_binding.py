"""ctypes binding of libpargeo_hip.so.

Argument marshalling only: tensors are passed as device pointers together
with torch's current HIP stream; every step of the computation runs in the
library's kernels.  There is no CPU fallback: without the built library or
without a GPU these functions raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libpargeo_hip.so")

PG_INT32, PG_FLOAT32 = 0, 1
_STATUS = {0: "PG_OK", 1: "PG_ERR_INVALID", 2: "PG_ERR_RANGE", 3: "PG_ERR_NOMEM",
           4: "PG_ERR_DEVICE", 5: "PG_ERR_UNSUPPORTED"}


class PargeoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class RangeError(PargeoError, ValueError):
    pass


_lib = None

vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
P64 = ctypes.POINTER(ctypes.c_int64)
P32 = ctypes.POINTER(ctypes.c_int32)

# name -> (restype, argtypes); the declarations of include/pargeo_hip.h
class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                           ctypes.c_void_p)),
                ("release", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)),
                ("ctx", ctypes.c_void_p)]


SIGNATURES = {
    "pg_set_allocator": (i32, [ctypes.POINTER(Allocator)]),
    "pg_release_cached": (i32, []),
    "pg_last_error": (ctypes.c_char_p, []),
    "pg_version": (ctypes.c_char_p, []),
    "pg_kdtree_build": (i32, [vp, i64, i32, i32, i32, vp, ctypes.POINTER(vp)]),
    "pg_kdtree_build_spatial": (i32, [vp, i64, i32, i32, i32, i32, vp, ctypes.POINTER(vp)]),
    "pg_tree_split_dims": (i32, [vp, vp, vp]),
    "pg_tree_offsets": (i32, [vp, vp, vp]),
    "pg_knn": (i32, [vp, vp, i64, i32, vp, vp, vp]),
    "pg_knn_noalloc": (i32, [vp, vp, i64, i32, vp, vp, vp]),
    "pg_knn_all": (i32, [vp, i32, vp, vp, vp]),
    "pg_knn_graph": (i32, [vp, i32, vp, vp, vp]),
    "pg_tree_info": (i32, [vp, P64, P32, P32, P32, P32]),
    "pg_tree_export": (i32, [vp, vp, vp, vp]),
    "pg_tree_nodes": (i32, [vp, P64, P64]),
    "pg_wspd": (i32, [vp, ctypes.c_double, vp, i64, P64, vp]),
    "pg_tree_export_nodes": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp]),
    "pg_tree_free": (None, [vp]),
    "pg_range_count": (i32, [vp, vp, i64, vp, vp, P64, vp]),
    "pg_range_report": (i32, [vp, vp, i64, vp, vp, i64, vp]),
    "pg_range_search": (i32, [vp, vp, i64, vp, vp, vp, i64, P64, vp]),
    "pg_bdl_create": (i32, [i32, i32, i32, i64, ctypes.POINTER(vp)]),
    "pg_bdl_create_spatial": (i32, [i32, i32, i32, i64, ctypes.POINTER(vp)]),
    "pg_bdl_insert": (i32, [vp, vp, i64, vp, P64]),
    "pg_bdl_erase": (i32, [vp, vp, i64, vp, P64]),
    "pg_bdl_knn": (i32, [vp, vp, i64, i32, vp, vp, vp]),
    "pg_bdl_size": (i64, [vp]),
    "pg_bdl_stats": (i32, [vp, P64, P64, P64, i32]),
    "pg_bdl_free": (None, [vp]),
    "pg_b1_create": (i32, [i32, i32, i32, ctypes.POINTER(vp)]),
    "pg_b1_create_spatial": (i32, [i32, i32, i32, ctypes.POINTER(vp)]),
    "pg_b1_insert": (i32, [vp, vp, i64, vp, P64]),
    "pg_b1_erase": (i32, [vp, vp, i64, vp, P64]),
    "pg_b1_knn": (i32, [vp, vp, i64, i32, vp, vp, vp]),
    "pg_b1_size": (i64, [vp]),
    "pg_b1_free": (None, [vp]),
    "pg_b2_create": (i32, [vp, i64, i32, i32, i32, vp, ctypes.POINTER(vp)]),
    "pg_b2_create_spatial": (i32, [vp, i64, i32, i32, i32, vp, ctypes.POINTER(vp)]),
    "pg_b2_insert": (i32, [vp, vp, i64, vp, P64]),
    "pg_b2_erase": (i32, [vp, vp, i64, vp, P64]),
    "pg_b2_knn": (i32, [vp, vp, i64, i32, vp, vp, vp]),
    "pg_b2_size": (i64, [vp]),
    "pg_b2_stats": (i32, [vp, P64, P32]),
    "pg_b2_free": (None, [vp]),
    "pg_batch_workspace": (i32, [P64, i32, i32, vp, ctypes.POINTER(ctypes.c_size_t)]),
    "pg_batch_create": (i32, [P64, i32, i32, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
    "pg_batch_knn_self": (i32, [vp, vp, i32, vp, vp, vp]),
    "pg_batch_knn": (i32, [vp, vp, vp, P64, i32, vp, vp, vp]),
    "pg_batch_check": (i32, [vp, i64, i32, vp]),
    "pg_batch_status": (i32, [vp, vp, P32]),
    "pg_batch_autotune": (i32, [vp, P64, i32, i32, i32, vp, vp]),
    "pg_batch_free": (None, [vp]),
    "pg_knn_backward": (i32, [vp, vp, i64, i64, i32, i32, vp, vp, vp, vp, vp]),
    "pg_knn_backward_atomic": (i32, [vp, vp, i64, i64, i32, i32, vp, vp, vp, vp, vp]),
    "pg_batch_backward": (i32, [vp, vp, i32, vp, vp, vp, vp, vp]),
}


KLIST_VGPR, KLIST_LDS = 1, 2


class Tune(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("lane_queries", ctypes.c_int32), ("klist", ctypes.c_int32)]


def lib():
    """Loads the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise RuntimeError(f"{SO} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(SO)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != 0:
        msg = lib().pg_last_error().decode()
        if status == 2:
            raise RangeError(status, msg)
        raise PargeoError(status, msg)


def stream_ptr(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.int32:
        return PG_INT32
    if t.dtype == torch.float32:
        return PG_FLOAT32
    raise TypeError(f"coordinates must be int32 or float32, got {t.dtype}")


def _points(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dim() != 2:
        raise ValueError(f"{name} must be [count][d]")
    return t.contiguous()


def _dist_dtype(code: int):
    return torch.int64 if code == PG_INT32 else torch.float32


class KdTree:
    """Static kd-tree on the GPU (object-median splits, leaves of at most
    ``leaf`` points).  Built by :func:`kdtree_build`."""

    def __init__(self, handle, points_dtype: int, device):
        self._h = handle
        self.dtype_code = points_dtype
        self.device = device
        n, d, leaf, levels, dt = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().pg_tree_info(self._h, ctypes.byref(n), ctypes.byref(d), ctypes.byref(leaf),
                                 ctypes.byref(levels), ctypes.byref(dt)))
        self.n, self.d, self.leaf, self.levels = n.value, d.value, leaf.value, levels.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pg_tree_free(h)
            self._h = None

    def knn(self, queries: torch.Tensor, k: int):
        """k nearest (distance, row) of each query: (idx int32 [m][k],
        dist int64 or float32 [m][k])."""
        q = _points(queries, "queries")
        if _dtype_code(q) != self.dtype_code:
            raise TypeError("queries must have the tree's dtype")
        m = q.shape[0]
        idx = torch.empty((m, k), dtype=torch.int32, device=q.device)
        dist = torch.empty((m, k), dtype=_dist_dtype(self.dtype_code), device=q.device)
        check(lib().pg_knn(self._h, ctypes.c_void_p(q.data_ptr()), m, k,
                           ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                           stream_ptr(q.device)))
        return idx, dist

    def knn_noalloc(self, queries: torch.Tensor, k: int, out):
        """As :meth:`knn`, through pg_knn_noalloc, into the caller's tensors
        out = (idx int32 [m][k], dist [m][k]); the library allocates no
        device memory (m <= 2^22)."""
        q = _points(queries, "queries")
        if _dtype_code(q) != self.dtype_code:
            raise TypeError("queries must have the tree's dtype")
        idx, dist = out
        m = q.shape[0]
        if (tuple(idx.shape) != (m, k) or tuple(dist.shape) != (m, k) or idx.dtype != torch.int32
                or dist.dtype != _dist_dtype(self.dtype_code) or not idx.is_contiguous()
                or not dist.is_contiguous()):
            raise ValueError("out must be contiguous (int32 [m][k], distance dtype [m][k])")
        check(lib().pg_knn_noalloc(self._h, ctypes.c_void_p(q.data_ptr()), m, k,
                                   ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                                   stream_ptr(q.device)))
        return idx, dist

    def knn_all(self, k: int, out=None):
        """All-points k-NN; row i belongs to input row i."""
        if out is None:
            idx = torch.empty((self.n, k), dtype=torch.int32, device=self.device)
            dist = torch.empty((self.n, k), dtype=_dist_dtype(self.dtype_code), device=self.device)
        else:
            idx, dist = out
        check(lib().pg_knn_all(self._h, k, ctypes.c_void_p(idx.data_ptr()),
                               ctypes.c_void_p(dist.data_ptr()), stream_ptr(self.device)))
        return idx, dist

    def knn_graph(self, k: int, out=None):
        """k-NN graph: row i holds the k nearest points other than input
        row i itself (directed edges i -> idx[i][r]), as (idx, dist)."""
        if out is None:
            idx = torch.empty((self.n, k), dtype=torch.int32, device=self.device)
            dist = torch.empty((self.n, k), dtype=_dist_dtype(self.dtype_code), device=self.device)
        else:
            idx, dist = out
        check(lib().pg_knn_graph(self._h, k, ctypes.c_void_p(idx.data_ptr()),
                                 ctypes.c_void_p(dist.data_ptr()), stream_ptr(self.device)))
        return idx, dist

    def _boxes(self, boxes):
        b = boxes.contiguous()
        if b.dim() != 3 or b.shape[1] != 2 or b.shape[2] != self.d:
            raise ValueError(f"boxes must be [m][2][{self.d}] (lo, hi)")
        if not b.is_cuda:
            raise ValueError("boxes must be a GPU tensor")
        if _dtype_code(b) != self.dtype_code:
            raise TypeError("boxes must have the tree's dtype")
        return b

    def range_count(self, boxes: torch.Tensor, offsets: bool = False):
        """Number of points in each closed box (boxes [m][2][d]: lo, hi) as
        int32 [m]; with ``offsets`` also the int64 [m+1] exclusive prefix sum
        and the total."""
        b = self._boxes(boxes)
        m = b.shape[0]
        counts = torch.empty(m, dtype=torch.int32, device=b.device)
        if not offsets:
            check(lib().pg_range_count(self._h, ctypes.c_void_p(b.data_ptr()), m,
                                       ctypes.c_void_p(counts.data_ptr()), None, None,
                                       stream_ptr(b.device)))
            return counts
        off = torch.empty(m + 1, dtype=torch.int64, device=b.device)
        total = ctypes.c_int64()
        check(lib().pg_range_count(self._h, ctypes.c_void_p(b.data_ptr()), m,
                                   ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(off.data_ptr()),
                                   ctypes.byref(total), stream_ptr(b.device)))
        return counts, off, total.value

    def range_report(self, boxes: torch.Tensor, offsets: torch.Tensor, out: torch.Tensor):
        """Writes the input rows of box i's points to out[offsets[i]:], in
        leaf order (the layout :meth:`range_count` gives)."""
        b = self._boxes(boxes)
        if offsets.dtype != torch.int64 or not offsets.is_contiguous() or offsets.numel() < b.shape[0]:
            raise ValueError("offsets must be a contiguous int64 tensor of at least m entries")
        if out.dtype != torch.int32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor")
        check(lib().pg_range_report(self._h, ctypes.c_void_p(b.data_ptr()), b.shape[0],
                                    ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    out.numel(), stream_ptr(b.device)))
        return out

    def range_search(self, boxes: torch.Tensor, capacity: int = None):
        """Range search: (offsets int64 [m+1], rows int32 [total]); box i's
        points are rows[offsets[i]:offsets[i+1]], in leaf order.  One call
        does both passes when the rows fit ``capacity`` (default: a guess
        from earlier calls on this tree); otherwise the rows buffer is sized
        from the counts and the reporting pass runs again."""
        b = self._boxes(boxes)
        m = b.shape[0]
        if capacity is None:
            per = getattr(self, "_range_per_box", 16.0)
            capacity = int(per * 1.25 * m) + 1024
        off = torch.empty(m + 1, dtype=torch.int64, device=b.device)
        out = torch.empty(max(capacity, 1), dtype=torch.int32, device=b.device)
        total = ctypes.c_int64()
        st = lib().pg_range_search(self._h, ctypes.c_void_p(b.data_ptr()), m, None,
                                   ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   capacity, ctypes.byref(total), stream_ptr(b.device))
        if m > 0:
            self._range_per_box = max(total.value / m, 1.0)
        if st != 0 and total.value > capacity:
            out = torch.empty(max(total.value, 1), dtype=torch.int32, device=b.device)
            self.range_report(b, off, out)
        else:
            check(st)
        return off, out[:total.value]

    def wspd(self, s: float = 2.0, capacity: int = None, out=None):
        """Well-separated pair decomposition (tree built with leaf 1): int32
        [P][2] heap node pairs on the device.  One call when the pairs fit
        ``capacity`` (default: ``out``'s rows, else a guess from the point
        count), else a second with the exact size."""
        if out is not None:
            capacity = out.shape[0] if capacity is None else capacity
        if capacity is None:
            capacity = 24 * self.n + 1024
        if out is None or out.shape[0] < capacity:
            out = torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=self.device)
        cnt = ctypes.c_int64()
        st = lib().pg_wspd(self._h, float(s), ctypes.c_void_p(out.data_ptr()), capacity,
                           ctypes.byref(cnt), stream_ptr(self.device))
        if st != 0 and cnt.value > capacity:
            out = torch.empty((max(cnt.value, 1), 2), dtype=torch.int32, device=self.device)
            st = lib().pg_wspd(self._h, float(s), ctypes.c_void_p(out.data_ptr()), cnt.value,
                               ctypes.byref(cnt), stream_ptr(self.device))
        check(st)
        return out[:cnt.value]

    def counts(self):
        """(nodes, leaves) of the tree."""
        nodes, leaves = ctypes.c_int64(), ctypes.c_int64()
        check(lib().pg_tree_nodes(self._h, ctypes.byref(nodes), ctypes.byref(leaves)))
        return nodes.value, leaves.value

    def nodes(self):
        """An explicit-node tree (spatial-median splits) as NumPy arrays in
        its breadth-first numbering: dict with split (coordinate dtype; 0 for
        leaves), dim (int32, -1 for leaves), child (int64 first child, -1 for
        leaves), lo / hi (int64 leaf-order range), level (int32) and perm
        (int32 input rows in leaf order)."""
        import numpy as np
        N, _ = self.counts()
        out = dict(split=np.empty(N, dtype=np.int32 if self.dtype_code == PG_INT32 else np.float32),
                   dim=np.empty(N, dtype=np.int32), child=np.empty(N, dtype=np.int64),
                   lo=np.empty(N, dtype=np.int64), hi=np.empty(N, dtype=np.int64),
                   level=np.empty(N, dtype=np.int32), perm=np.empty(self.n, dtype=np.int32))
        check(lib().pg_tree_export_nodes(self._h, *[ctypes.c_void_p(out[k].ctypes.data) for k in
                                                     ("split", "dim", "child", "lo", "hi", "level",
                                                      "perm")], stream_ptr(self.device)))
        return out

    def offsets(self):
        """Leaf offsets (NumPy int64 [leaves + 1])."""
        import numpy as np
        loff = np.empty(self.counts()[1] + 1, dtype=np.int64)
        check(lib().pg_tree_offsets(self._h, ctypes.c_void_p(loff.ctypes.data), stream_ptr(self.device)))
        return loff

    def split_dims(self):
        """Split dimension of every internal heap node (NumPy uint8 [2^L],
        index 0 unused)."""
        import numpy as np
        dims = np.empty(1 << self.levels, dtype=np.uint8)
        check(lib().pg_tree_split_dims(self._h, ctypes.c_void_p(dims.ctypes.data), stream_ptr(self.device)))
        return dims

    def export(self):
        """(split values of heap nodes 1..2^L-1, input rows in leaf order) as
        NumPy arrays."""
        import numpy as np
        ni = (1 << self.levels) - 1
        splits = np.empty(ni, dtype=np.int32 if self.dtype_code == PG_INT32 else np.float32)
        perm = np.empty(self.n, dtype=np.int32)
        check(lib().pg_tree_export(self._h, ctypes.c_void_p(splits.ctypes.data),
                                   ctypes.c_void_p(perm.ctypes.data), stream_ptr(self.device)))
        return splits, perm


def kdtree_build(points: torch.Tensor, leaf: int = 16, split: str = "object",
                 dim_rule: str = "cycle", space: str = "cell") -> KdTree:
    """Builds a kd-tree: ``split="object"`` (object median, every leaf at most
    ``leaf`` points) or ``"spatial"`` (spaces cut at their midpoints until a
    node holds at most ``leaf`` points or only identical ones, any depth;
    ``dim_rule`` "cycle" = depth mod d, "widest" = the space's widest side;
    ``space`` "cell" = the node's cell, "points" = the bounding box of the
    node's points)."""
    p = _points(points, "points")
    code = _dtype_code(p)
    h = ctypes.c_void_p()
    args = (ctypes.c_void_p(p.data_ptr()), p.shape[0], p.shape[1], leaf, code)
    if space not in ("cell", "points"):
        raise ValueError("space must be 'cell' or 'points'")
    if split == "object":
        if dim_rule != "cycle" or space != "cell":
            raise ValueError("object-median trees cycle through the dimensions")
        check(lib().pg_kdtree_build(*args, stream_ptr(p.device), ctypes.byref(h)))
    elif split == "spatial":
        rule = {"cycle": 0, "widest": 1}[dim_rule] | (2 if space == "points" else 0)
        check(lib().pg_kdtree_build_spatial(*args, rule, stream_ptr(p.device), ctypes.byref(h)))
    else:
        raise ValueError("split must be 'object' or 'spatial'")
    return KdTree(h, code, p.device)


def _dynamic_split(split: str) -> str:
    if split not in ("object", "spatial"):
        raise ValueError("split must be 'object' or 'spatial'")
    return "_spatial" if split == "spatial" else ""


class BDLTree:
    """Batch-dynamic kd-tree (Section 5): insert / erase batches, k-NN over the
    live points.  Ids are a global insertion counter.  ``split`` picks object-
    or spatial-median static trees (Section 6.3 runs both)."""

    def __init__(self, d: int, dtype=torch.int32, leaf: int = 16, X: int = 1 << 14,
                 device="cuda", split: str = "object"):
        self.d, self.leaf, self.X = d, leaf, X
        self.dtype = dtype
        self.code = PG_INT32 if dtype == torch.int32 else PG_FLOAT32
        self.device = torch.device(device)
        h = ctypes.c_void_p()
        fn = getattr(lib(), "pg_bdl_create" + _dynamic_split(split))
        check(fn(d, self.code, leaf, X, ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pg_bdl_free(h)
            self._h = None

    def _rows(self, pts):
        p = _points(pts, "points")
        if p.shape[1] != self.d or _dtype_code(p) != self.code:
            raise TypeError("points must be [m][d] of the tree's dtype")
        return p

    def insert(self, pts) -> int:
        p = self._rows(pts)
        first = ctypes.c_int64()
        check(lib().pg_bdl_insert(self._h, ctypes.c_void_p(p.data_ptr()), p.shape[0],
                                  stream_ptr(p.device), ctypes.byref(first)))
        return first.value

    def erase(self, pts) -> int:
        p = self._rows(pts)
        cnt = ctypes.c_int64()
        check(lib().pg_bdl_erase(self._h, ctypes.c_void_p(p.data_ptr()), p.shape[0],
                                 stream_ptr(p.device), ctypes.byref(cnt)))
        return cnt.value

    def knn(self, queries, k: int, out=None):
        q = self._rows(queries)
        m = q.shape[0]
        if out is None:
            ids = torch.empty((m, k), dtype=torch.int64, device=q.device)
            dist = torch.empty((m, k), dtype=_dist_dtype(self.code), device=q.device)
        else:
            ids, dist = out
        check(lib().pg_bdl_knn(self._h, ctypes.c_void_p(q.data_ptr()), m, k,
                               ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                               stream_ptr(q.device)))
        return ids, dist

    def size(self) -> int:
        return lib().pg_bdl_size(self._h)

    def stats(self, max_trees: int = 64):
        F, b = ctypes.c_int64(), ctypes.c_int64()
        live = (ctypes.c_int64 * max_trees)()
        check(lib().pg_bdl_stats(self._h, ctypes.byref(F), ctypes.byref(b), live, max_trees))
        return F.value, b.value, list(live)


def _offsets_array(offsets):
    import numpy as np
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    return o, o.ctypes.data_as(P64)


class BatchKnn:
    """Per-cloud all-points k-NN of many float32 clouds in one persistent
    launch.  ``offsets`` (host, [C+1]) delimit the clouds in the point array.
    The plan (and a library-owned workspace) is made once; ``knn_self`` only
    launches, so it can be captured in a CUDA/HIP graph."""

    def __init__(self, offsets, d: int, leaf: int = 0, blocks_per_cu: int = 0,
                 lane_queries: int = 0, klist: int = 0, device="cuda"):
        self.offsets, optr = _offsets_array(offsets)
        self.C = len(self.offsets) - 1
        self.N = int(self.offsets[-1])
        self.d = d
        self.device = torch.device(device)
        self.tune = Tune(leaf, blocks_per_cu, lane_queries, klist)
        self.generation = 0  # knn_self calls so far (the trees belong to the last)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().pg_batch_create(optr, self.C, d, ctypes.byref(self.tune), None, 0,
                                        stream_ptr(self.device), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pg_batch_free(h)
            self._h = None

    def knn_self(self, points: torch.Tensor, k: int, out=None):
        p = _points(points, "points")
        if p.dtype != torch.float32 or p.shape != (self.N, self.d):
            raise TypeError("points must be float32 [N][d] matching the offsets")
        if out is None:
            idx = torch.empty((self.N, k), dtype=torch.int32, device=p.device)
            d2 = torch.empty((self.N, k), dtype=torch.float32, device=p.device)
        else:
            idx, d2 = out
        check(lib().pg_batch_knn_self(self._h, ctypes.c_void_p(p.data_ptr()), k,
                                      ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()),
                                      stream_ptr(p.device)))
        self.generation += 1
        return idx, d2

    def knn(self, points: torch.Tensor, queries: torch.Tensor, q_offsets, k: int, out=None):
        """k-NN of a separate query set per cloud (cloud c's queries are rows
        [q_offsets[c], q_offsets[c+1]) of ``queries``) in one persistent
        launch: (idx int32 [M][k] global point rows, d2 float32 [M][k])."""
        p = _points(points, "points")
        q = _points(queries, "queries")
        if p.dtype != torch.float32 or p.shape != (self.N, self.d):
            raise TypeError("points must be float32 [N][d] matching the offsets")
        qo, qptr = _offsets_array(q_offsets)
        if len(qo) != self.C + 1 or q.dtype != torch.float32 or q.shape != (int(qo[-1]), self.d):
            raise TypeError("queries must be float32 [M][d] with q_offsets of C + 1 entries")
        M = q.shape[0]
        if out is None:
            idx = torch.empty((M, k), dtype=torch.int32, device=p.device)
            d2 = torch.empty((M, k), dtype=torch.float32, device=p.device)
        else:
            idx, d2 = out
        check(lib().pg_batch_knn(self._h, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                                 qptr, k, ctypes.c_void_p(idx.data_ptr()),
                                 ctypes.c_void_p(d2.data_ptr()), stream_ptr(p.device)))
        self.generation += 1
        return idx, d2

    def backward(self, points: torch.Tensor, idx: torch.Tensor, d2: torch.Tensor,
                 grad_d2: torch.Tensor, out=None):
        """Gradient of sum grad_d2 * d2 w.r.t. the points for the last
        knn_self (see pg_batch_backward); deterministic."""
        p = _points(points, "points")
        k = idx.shape[1]
        idx = idx.contiguous()
        d2 = d2.contiguous()
        g = grad_d2.contiguous().to(torch.float32)
        gp = torch.empty_like(p) if out is None else out
        check(lib().pg_batch_backward(self._h, ctypes.c_void_p(p.data_ptr()), k,
                                      ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()),
                                      ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(gp.data_ptr()),
                                      stream_ptr(p.device)))
        return gp

    def flags(self) -> int:
        flag = ctypes.c_int32()
        check(lib().pg_batch_status(self._h, stream_ptr(self.device), ctypes.byref(flag)))
        return flag.value

    def timed_out(self) -> bool:
        """A wait of the last launch timed out."""
        return bool(self.flags() & 1)

    def backward_nonfinite(self) -> bool:
        """A backward met a cloud whose term bound is not a finite float (its
        gradients are NaN)."""
        return bool(self.flags() & 2)


def batch_check(points: torch.Tensor):
    p = _points(points, "points")
    check(lib().pg_batch_check(ctypes.c_void_p(p.data_ptr()), p.shape[0], p.shape[1],
                               stream_ptr(p.device)))


def batch_autotune(points: torch.Tensor, offsets, k: int):
    p = _points(points, "points")
    o, optr = _offsets_array(offsets)
    t = Tune()
    check(lib().pg_batch_autotune(ctypes.c_void_p(p.data_ptr()), optr, len(o) - 1, p.shape[1], k,
                                  stream_ptr(p.device), ctypes.byref(t)))
    return {"leaf": t.leaf, "blocks_per_cu": t.blocks_per_cu, "lane_queries": t.lane_queries,
            "klist": t.klist}


def knn_backward(queries, points, idx, grad_d2, grad_q=None, grad_p=None, self_mode=False,
                 deterministic=True):
    """Gradients of sum g * D with fixed neighbours (see pg_knn_backward).
    self_mode: queries is points, one gradient array receives both roles.
    deterministic=False: float atomics for the point gradients
    (pg_knn_backward_atomic; equal up to rounding, not bit-reproducible)."""
    q = _points(queries, "queries")
    x = _points(points, "points")
    idx = idx.contiguous()
    g = grad_d2.contiguous().to(torch.float32)
    m, d = q.shape
    n = x.shape[0]
    k = idx.shape[1]
    if self_mode:
        gq = torch.empty_like(x) if grad_q is None else grad_q
        gp = gq
    else:
        gq = torch.empty_like(q) if grad_q is None else grad_q
        gp = torch.empty_like(x) if grad_p is None else grad_p
    fn = lib().pg_knn_backward if deterministic else lib().pg_knn_backward_atomic
    check(fn(ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(x.data_ptr()), m, n,
             d, k, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(g.data_ptr()),
             ctypes.c_void_p(gq.data_ptr()), ctypes.c_void_p(gp.data_ptr()),
             stream_ptr(q.device)))
    return gq, gp


class B2Tree:
    """The second baseline of Section 6.3: one kd-tree over the initial
    points whose splits never change; inserts join the leaf they reach,
    erases leave tombstones.  Same interface as :class:`BDLTree`."""

    def __init__(self, points: torch.Tensor, leaf: int = 16, split: str = "object"):
        p = _points(points, "points")
        self.d, self.leaf = p.shape[1], leaf
        self.code = _dtype_code(p)
        self.device = p.device
        h = ctypes.c_void_p()
        fn = getattr(lib(), "pg_b2_create" + _dynamic_split(split))
        check(fn(ctypes.c_void_p(p.data_ptr()), p.shape[0], self.d, leaf, self.code,
                 stream_ptr(p.device), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pg_b2_free(h)
            self._h = None

    def _rows(self, pts):
        p = _points(pts, "points")
        if p.shape[1] != self.d or _dtype_code(p) != self.code:
            raise TypeError("points must be [m][d] of the tree's dtype")
        return p

    def insert(self, pts) -> int:
        p = self._rows(pts)
        first = ctypes.c_int64()
        check(lib().pg_b2_insert(self._h, ctypes.c_void_p(p.data_ptr()), p.shape[0],
                                 stream_ptr(p.device), ctypes.byref(first)))
        return first.value

    def erase(self, pts) -> int:
        p = self._rows(pts)
        cnt = ctypes.c_int64()
        check(lib().pg_b2_erase(self._h, ctypes.c_void_p(p.data_ptr()), p.shape[0],
                                stream_ptr(p.device), ctypes.byref(cnt)))
        return cnt.value

    def knn(self, queries, k: int, out=None):
        q = self._rows(queries)
        m = q.shape[0]
        if out is None:
            ids = torch.empty((m, k), dtype=torch.int64, device=q.device)
            dist = torch.empty((m, k), dtype=_dist_dtype(self.code), device=q.device)
        else:
            ids, dist = out
        check(lib().pg_b2_knn(self._h, ctypes.c_void_p(q.data_ptr()), m, k,
                              ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                              stream_ptr(q.device)))
        return ids, dist

    def size(self) -> int:
        return lib().pg_b2_size(self._h)

    def stats(self):
        stored, levels = ctypes.c_int64(), ctypes.c_int32()
        check(lib().pg_b2_stats(self._h, ctypes.byref(stored), ctypes.byref(levels)))
        return stored.value, levels.value


class B1Tree:
    """The first baseline of Section 6.3: one static kd-tree over the live
    points, rebuilt from scratch after every batch.  Same interface as
    :class:`BDLTree`."""

    def __init__(self, d: int, dtype=torch.int32, leaf: int = 16, device="cuda",
                 split: str = "object"):
        self.d, self.leaf = d, leaf
        self.code = PG_INT32 if dtype == torch.int32 else PG_FLOAT32
        self.device = torch.device(device)
        h = ctypes.c_void_p()
        fn = getattr(lib(), "pg_b1_create" + _dynamic_split(split))
        check(fn(d, self.code, leaf, ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pg_b1_free(h)
            self._h = None

    _rows = B2Tree._rows

    def insert(self, pts) -> int:
        p = self._rows(pts)
        first = ctypes.c_int64()
        check(lib().pg_b1_insert(self._h, ctypes.c_void_p(p.data_ptr()), p.shape[0],
                                 stream_ptr(p.device), ctypes.byref(first)))
        return first.value

    def erase(self, pts) -> int:
        p = self._rows(pts)
        cnt = ctypes.c_int64()
        check(lib().pg_b1_erase(self._h, ctypes.c_void_p(p.data_ptr()), p.shape[0],
                                stream_ptr(p.device), ctypes.byref(cnt)))
        return cnt.value

    def knn(self, queries, k: int, out=None):
        q = self._rows(queries)
        m = q.shape[0]
        if out is None:
            ids = torch.empty((m, k), dtype=torch.int64, device=q.device)
            dist = torch.empty((m, k), dtype=_dist_dtype(self.code), device=q.device)
        else:
            ids, dist = out
        check(lib().pg_b1_knn(self._h, ctypes.c_void_p(q.data_ptr()), m, k,
                              ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                              stream_ptr(q.device)))
        return ids, dist

    def size(self) -> int:
        return lib().pg_b1_size(self._h)


_torch_allocator = None


def release_cached():
    """Returns the device blocks the library's default allocator keeps for
    reuse to the device (pg_release_cached; synchronises the device)."""
    check(lib().pg_release_cached())


def use_torch_allocator(enable: bool = True):
    """Routes the library's device allocations through torch's caching
    allocator (pg_set_allocator), or back to the library's own pool."""
    global _torch_allocator
    if not enable:
        check(lib().pg_set_allocator(None))
        _torch_allocator = None
        return
    A = Allocator._fields_

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:
            return None

    def _release(p, stream, ctx):
        torch.cuda.caching_allocator_delete(p)

    a = Allocator(A[0][1](_alloc), A[1][1](_release), None)
    check(lib().pg_set_allocator(ctypes.byref(a)))
    _torch_allocator = a  # keep the callbacks alive
