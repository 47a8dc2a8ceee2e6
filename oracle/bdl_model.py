"""BDL-tree model -- TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

The logarithmic method of Section 5 ("Parallel Batch Insertion") and
Appendix C (Algorithm 3, batch insertion; Algorithm 4, batch deletion),
replayed on plain point sets: static tree i holds at most X * 2^i points,
the buffer holds fewer than X, F is the bitmask of non-empty static trees.
No kd-tree is needed to model which points live where; k-NN over the live
set is delegated to the oracle's definition (``knn_brute``) or its kd-tree.

Readings adopted where the paper is silent:
  * F_new = F + floor(|P| / X) (the floor of Section 5's text);
  * |P| mod X points go to the buffer; when they would fill it, the buffer's
    points plus enough batch points to make X join the tree-bound points;
  * bit i of F set  <=>  static tree i is non-empty;
  * each destroyed tree i moves whole into the smallest new tree j > i;
    tree-bound points fill new trees in ascending j, the old buffer's points
    first, then batch points in batch order; the last batch points form the
    new buffer;
  * a tree keeps its points in the order they were staged for it (destroyed
    trees' live points in ascending tree index, each in its own staging
    order, then the fresh points); the gathered set R of Algorithm 4 uses the
    same order;
  * erase removes every live point whose coordinates equal an erase point
    (absent points are no-ops) from every static tree and from the buffer;
  * a static tree is gathered into R when its live count < X * 2^i / 2; the
    buffer is exempt.
"""
from __future__ import annotations

import numpy as np


def insert_plan(F: int, b: int, m: int, X: int):
    """Counts-only Algorithm 3 for a batch of m points.

    Returns dict(A, F_new, new, destroyed, assign, quota, to_buffer,
    buffer_after, overflow) where ``assign[j]`` lists the destroyed trees that
    move into new tree j and ``quota[j]`` the number of tree-bound points it
    takes."""
    r = m % X
    A = m // X
    overflow = b + r >= X
    if overflow:
        A += 1
        buffer_after = b + r - X
    else:
        buffer_after = b + r
    F_new = F + A
    new = F_new & ~F
    destroyed = F & ~F_new
    assign, quota = {}, {}
    new_bits = [j for j in range(F_new.bit_length()) if (new >> j) & 1]
    for i in range(F.bit_length()):
        if (destroyed >> i) & 1:
            j = min(t for t in new_bits if t > i)
            assign.setdefault(j, []).append(i)
    for j in new_bits:
        quota[j] = (1 << j) * X - sum((1 << i) * X for i in assign.get(j, []))
    return dict(A=A, F_new=F_new, new=new, destroyed=destroyed, assign=assign,
                quota=quota, buffer_after=buffer_after, overflow=overflow,
                to_buffer=r if not overflow else buffer_after)


def _canonical_bits(a):
    """The 32-bit patterns of the coordinates of a, -0.0 first made +0.0, so
    that two rows are equal coordinate by coordinate exactly when their
    patterns are."""
    a = np.ascontiguousarray(a)
    if a.dtype.kind == "f":
        a = np.where(a == 0, np.zeros((), a.dtype), a)
    return np.ascontiguousarray(a).view(np.uint32).reshape(a.shape)


def rows_in(a, b):
    """Boolean mask over the rows of a: the row equals some row of b."""
    A, B = _canonical_bits(a), _canonical_bits(b)
    d = A.shape[1]
    if len(A) == 0 or len(B) == 0:
        return np.zeros(len(A), dtype=bool)
    # candidates by the first two coordinates (one 64-bit key), then the
    # whole rows of the candidates as byte strings
    def pre(x):
        k = x[:, 0].astype(np.uint64) << np.uint64(32)
        return k | x[:, 1].astype(np.uint64) if d > 1 else k
    cand = np.isin(pre(A), pre(B))
    if d <= 2:
        return cand
    whole = lambda x: np.ascontiguousarray(x).view(np.dtype((np.void, 4 * d))).ravel()
    out = np.zeros(len(A), dtype=bool)
    ci = np.nonzero(cand)[0]
    out[ci] = np.isin(whole(A[ci]), whole(B))
    return out


class BDLModel:
    """Point-set model of the BDL-tree.  Point ids are a global insertion
    counter starting at 0.  Trees and the buffer are id arrays in staging
    order."""

    def __init__(self, d: int, X: int, dtype=np.int32):
        self.d, self.X, self.dtype = d, X, np.dtype(dtype)
        self.coords = np.zeros((0, d), dtype=self.dtype)  # indexed by id
        self.alive = np.zeros(0, dtype=bool)
        self.trees: dict[int, np.ndarray] = {}           # i -> ids in staging order
        self.buffer = np.zeros(0, dtype=np.int64)
        self.next_id = 0

    # -- state ------------------------------------------------------------
    def F(self) -> int:
        f = 0
        for i, ids in self.trees.items():
            if len(ids):
                f |= 1 << i
        return f

    def tree_live(self, i: int) -> int:
        ids = self.trees.get(i)
        return int(np.count_nonzero(self.alive[ids])) if ids is not None and len(ids) else 0

    def stats(self, max_trees: int = 64):
        live = [self.tree_live(i) for i in range(max_trees)]
        return self.F(), len(self.buffer), live

    def size(self) -> int:
        return int(np.count_nonzero(self.alive))

    def live(self):
        ids = np.nonzero(self.alive)[0].astype(np.int64)
        return self.coords[ids], ids

    # -- Algorithm 3 --------------------------------------------------------
    def _insert_ids(self, S):
        S = np.asarray(S, dtype=np.int64)
        X = self.X
        F = self.F()
        plan = insert_plan(F, len(self.buffer), len(S), X)
        m, r = len(S), len(S) % X
        if plan["overflow"]:
            take = X - len(self.buffer)
            n_fresh = (m // X) * X + take
            bound = np.concatenate([self.buffer, S[:n_fresh]])
            self.buffer = S[n_fresh:].copy()
        else:
            bound = S[:m - r]
            self.buffer = np.concatenate([self.buffer, S[m - r:]])
        if plan["A"] == 0:
            return plan
        pos = 0
        new_trees = {}
        for j in sorted(plan["quota"]):
            members = []
            for i in sorted(plan["assign"].get(j, [])):
                ids = self.trees[i]
                members.append(ids[self.alive[ids]])
            q = plan["quota"][j]
            members.append(bound[pos:pos + q])
            pos += q
            new_trees[j] = np.concatenate(members)
        assert pos == len(bound)
        for i in range(F.bit_length()):
            if (plan["destroyed"] >> i) & 1:
                self.trees[i] = np.zeros(0, dtype=np.int64)
        for j, members in new_trees.items():
            self.trees[j] = members
        return plan

    def insert(self, pts) -> int:
        pts = np.ascontiguousarray(pts, dtype=self.dtype).reshape(-1, self.d)
        m = len(pts)
        first = self.next_id
        self.coords = np.concatenate([self.coords, pts])
        self.alive = np.concatenate([self.alive, np.ones(m, dtype=bool)])
        self.next_id += m
        self._insert_ids(np.arange(first, first + m, dtype=np.int64))
        return first

    # -- Algorithm 4 --------------------------------------------------------
    def erase(self, pts) -> int:
        pts = np.ascontiguousarray(pts, dtype=self.dtype).reshape(-1, self.d)
        if len(pts) == 0:
            return 0
        live_ids = np.nonzero(self.alive)[0]
        hit = live_ids[rows_in(self.coords[live_ids], pts)]
        self.alive[hit] = False
        self.buffer = self.buffer[self.alive[self.buffer]]
        R = []
        for i in sorted(self.trees):
            ids = self.trees[i]
            if not len(ids):
                continue
            live_i = ids[self.alive[ids]]
            if 2 * len(live_i) < self.X * (1 << i):
                R.append(live_i)
                self.trees[i] = np.zeros(0, dtype=np.int64)
        if R:
            self._insert_ids(np.concatenate(R))
        return len(hit)
