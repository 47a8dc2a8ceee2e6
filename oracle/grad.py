"""Gradient oracle -- TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

Loss = sum over (i, r) of g[i, r] * D(q_i, x_{idx[i, r]}), D the squared
Euclidean distance, with the neighbour sets idx held fixed.  Its gradient,
written out in FP64:

    dL/dq_i = sum_r 2 g[i,r] (q_i - x_j),          j = idx[i, r]
    dL/dx_j = - sum over (i, r) with idx[i, r] = j of 2 g[i,r] (q_i - x_j)

Central differences re-run the whole k-NN (the definition, in FP64)
at +-h, so that they include any change of the neighbour lists; coordinates
whose perturbation changes a list (its set or the order of its ranks) are
reported, and are excluded from comparisons ("away from ties").
"""
from __future__ import annotations

import numpy as np


def grad_closed_form(q, x, idx, g):
    q = np.asarray(q, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    g = np.asarray(g, dtype=np.float64)
    gq = np.zeros_like(q)
    gx = np.zeros_like(x)
    m, k = idx.shape
    for i in range(m):
        for r in range(k):
            j = idx[i, r]
            if j < 0:
                continue
            diff = q[i] - x[j]
            gq[i] += 2.0 * g[i, r] * diff
            gx[j] -= 2.0 * g[i, r] * diff
    return gq, gx


def loss_fixed(q, x, idx, g):
    """sum g * D with the given neighbour sets, FP64."""
    q = np.asarray(q, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    tot = 0.0
    m, k = idx.shape
    for i in range(m):
        for r in range(k):
            j = idx[i, r]
            if j >= 0:
                tot += g[i, r] * float(np.sum((q[i] - x[j]) ** 2))
    return tot


def fd_self(points, k, g, h=1e-6):
    """Central differences of L(P) = sum_{i,r} g[i,r] D(p_i, p_{idx[i,r]})
    where queries and data are the same point set P and the neighbour sets
    are recomputed from the perturbed points in FP64.

    Returns (grad [n][d], stable mask [n][d]) where stable marks coordinates
    whose perturbation changed no neighbour list.  The weights g[i, r] belong
    to ranks, so a swap of two ranks inside a list is a tie (a kink of the
    loss) just as a change of the set is; the lists are compared in order."""
    P = np.asarray(points, dtype=np.float64)
    n, d = P.shape
    base = _sets64(P, k)
    grad = np.zeros_like(P)
    stable = np.ones_like(P, dtype=bool)
    for a in range(n):
        for c in range(d):
            vals = []
            for s in (+1.0, -1.0):
                Pp = P.copy()
                Pp[a, c] += s * h
                ids = _sets64(Pp, k)
                if not np.array_equal(ids, base):
                    stable[a, c] = False
                vals.append(_loss_sets(Pp, ids, g))
            grad[a, c] = (vals[0] - vals[1]) / (2.0 * h)
    return grad, stable


def _sets64(P, k):
    """k-NN sets of every row of P among the rows of P, in exact FP64 (ties to
    the smaller index) -- the definition, vectorised for small n."""
    diff = P[:, None, :] - P[None, :, :]
    D = np.sum(diff * diff, axis=2)
    n = P.shape[0]
    order = np.lexsort((np.broadcast_to(np.arange(n), (n, n)), D), axis=1)
    return order[:, :k]


def _loss_sets(P, ids, g):
    tot = 0.0
    for i in range(P.shape[0]):
        diff = P[i] - P[ids[i]]
        tot += float(np.sum(g[i] * np.sum(diff * diff, axis=1)))
    return tot


def fd_self_incremental(points, k, g, h=1e-6):
    """fd_self with the same results, computed incrementally: perturbing
    point a changes only row and column a of the FP64 distance matrix, so
    only the neighbour lists that hold a, or that a's new distance now
    enters, are sorted again, and the loss is summed from the updated matrix.
    The lists of every other row, and every other distance, are those of the
    unperturbed points."""
    P = np.asarray(points, dtype=np.float64)
    n, d = P.shape
    g = np.asarray(g, dtype=np.float64)
    diff = P[:, None, :] - P[None, :, :]
    D = np.sum(diff * diff, axis=2)
    base = _lists(D, k)
    rows = np.arange(n)[:, None]
    kth_d = D[np.arange(n), base[:, k - 1]]
    kth_id = base[:, k - 1]
    holds = np.zeros((n, n), dtype=bool)
    holds[rows, base] = True  # holds[i, a]: a is in row i's list
    grad = np.zeros_like(P)
    stable = np.ones_like(P, dtype=bool)
    for a in range(n):
        for c in range(d):
            vals = []
            for s in (+1.0, -1.0):
                Pp = P.copy()
                Pp[a, c] += s * h
                da = Pp[a] - Pp
                ra = np.sum(da * da, axis=1)
                Dp = D.copy()
                Dp[a, :] = ra
                Dp[:, a] = ra
                hit = holds[:, a] | (ra < kth_d) | ((ra == kth_d) & (a < kth_id))
                hit[a] = True
                ids = base.copy()
                ids[hit] = _lists(Dp[hit], k)
                if not np.array_equal(ids, base):
                    stable[a, c] = False
                # row sums, then accumulated in row order (as _loss_sets)
                vals.append(float(np.cumsum(np.sum(g * Dp[rows, ids], axis=1))[-1]))
            grad[a, c] = (vals[0] - vals[1]) / (2.0 * h)
    return grad, stable


def _lists(Drows, k):
    """The k smallest (distance, column) keys of each row, as columns."""
    cols = np.broadcast_to(np.arange(Drows.shape[1]), Drows.shape)
    return np.lexsort((cols, Drows), axis=1)[:, :k]
