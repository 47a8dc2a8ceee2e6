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


class BDLModel:
    """Point-set model of the BDL-tree.  Point ids are a global insertion
    counter starting at 0."""

    def __init__(self, d: int, X: int, dtype=np.int32):
        self.d, self.X, self.dtype = d, X, np.dtype(dtype)
        self.coords = np.zeros((0, d), dtype=self.dtype)  # indexed by id
        self.alive = np.zeros(0, dtype=bool)
        self.trees: dict[int, list] = {}                 # i -> ids in staging order
        self.buffer: list = []
        self.next_id = 0

    # -- state ------------------------------------------------------------
    def F(self) -> int:
        f = 0
        for i, ids in self.trees.items():
            if ids:
                f |= 1 << i
        return f

    def tree_live(self, i: int) -> int:
        ids = self.trees.get(i, [])
        return int(np.count_nonzero(self.alive[np.asarray(ids, dtype=np.int64)])) if ids else 0

    def stats(self, max_trees: int = 64):
        live = [self.tree_live(i) for i in range(max_trees)]
        return self.F(), len(self.buffer), live

    def size(self) -> int:
        return int(np.count_nonzero(self.alive))

    def live(self):
        ids = np.nonzero(self.alive)[0].astype(np.int64)
        return self.coords[ids], ids

    # -- Algorithm 3 --------------------------------------------------------
    def _insert_ids(self, S: list):
        X = self.X
        F = self.F()
        plan = insert_plan(F, len(self.buffer), len(S), X)
        m, r = len(S), len(S) % X
        if plan["overflow"]:
            take = X - len(self.buffer)
            n_fresh = (m // X) * X + take
            bound = list(self.buffer) + list(S[:n_fresh])
            self.buffer = list(S[n_fresh:])
        else:
            bound = list(S[:m - r])
            self.buffer = self.buffer + list(S[m - r:])
        if plan["A"] == 0:
            return plan
        pos = 0
        new_trees = {}
        for j in sorted(plan["quota"]):
            members = []
            for i in sorted(plan["assign"].get(j, [])):
                members += [t for t in self.trees[i] if self.alive[t]]
            q = plan["quota"][j]
            members += bound[pos:pos + q]
            pos += q
            new_trees[j] = members
        assert pos == len(bound)
        for i in range(F.bit_length()):
            if (plan["destroyed"] >> i) & 1:
                self.trees[i] = []
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
        self._insert_ids(list(range(first, first + m)))
        return first

    # -- Algorithm 4 --------------------------------------------------------
    def erase(self, pts) -> int:
        pts = np.ascontiguousarray(pts, dtype=self.dtype).reshape(-1, self.d)
        if len(pts) == 0:
            return 0
        want = {tuple(p) for p in pts.tolist()}
        live_ids = np.nonzero(self.alive)[0]
        hit = [t for t, c in zip(live_ids.tolist(), self.coords[live_ids].tolist())
               if tuple(c) in want]
        self.alive[np.asarray(hit, dtype=np.int64)] = False
        self.buffer = [t for t in self.buffer if self.alive[t]]
        R = []
        for i in sorted(self.trees):
            ids = self.trees[i]
            if not ids:
                continue
            live_i = [t for t in ids if self.alive[t]]
            if 2 * len(live_i) < self.X * (1 << i):
                R += live_i
                self.trees[i] = []
        if R:
            self._insert_ids(R)
        return len(hit)
