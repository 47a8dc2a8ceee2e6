"""Differentiable k-NN squared distances (torch.autograd.Function).

Forward: the GPU k-NN (batched clouds in one persistent launch, or a static
tree for a separate query set).  Backward: the library's hand-written kernels
(pg_batch_backward in the clouds' leaf order while the forward's trees are
still current, else pg_knn_backward), with the neighbour sets held fixed from
the forward pass.
"""
from __future__ import annotations

import torch

from . import _binding as B


class _SelfKnn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, k, batch):
        idx, d2 = batch.knn_self(x.detach(), k)
        ctx.save_for_backward(x, idx, d2)
        ctx.batch = batch
        ctx.generation = batch.generation
        ctx.mark_non_differentiable(idx)
        return d2, idx

    @staticmethod
    def backward(ctx, g_d2, g_idx):
        x, idx, d2 = ctx.saved_tensors
        if g_d2 is None:
            return None, None, None
        if ctx.batch.generation == ctx.generation:
            # the clouds' trees of this forward are still in the workspace
            gx = ctx.batch.backward(x.detach(), idx, d2, g_d2)
        else:
            gx, _ = B.knn_backward(x.detach(), x.detach(), idx, g_d2, self_mode=True)
        return gx, None, None


class _BatchQueryKnn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, x, k, batch, q_offsets):
        idx, d2 = batch.knn(x.detach(), q.detach(), q_offsets, k)
        ctx.save_for_backward(q, x, idx)
        ctx.mark_non_differentiable(idx)
        return d2, idx

    @staticmethod
    def backward(ctx, g_d2, g_idx):
        q, x, idx = ctx.saved_tensors
        if g_d2 is None:
            return None, None, None, None, None
        gq, gx = B.knn_backward(q.detach(), x.detach(), idx, g_d2)
        return gq, gx, None, None, None


class _QueryKnn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, x, k, leaf):
        tree = B.kdtree_build(x.detach(), leaf=leaf)
        idx, d2 = tree.knn(q.detach(), k)
        ctx.save_for_backward(q, x, idx)
        ctx.mark_non_differentiable(idx)
        return d2, idx

    @staticmethod
    def backward(ctx, g_d2, g_idx):
        q, x, idx = ctx.saved_tensors
        if g_d2 is None:
            return None, None, None, None
        gq, gx = B.knn_backward(q.detach(), x.detach(), idx, g_d2)
        return gq, gx, None, None


def knn_sqdist(x: torch.Tensor, k: int, offsets=None, queries: torch.Tensor | None = None,
               batch: "B.BatchKnn | None" = None, leaf: int = 16, q_offsets=None):
    """k nearest squared distances and neighbour rows.

    * ``queries is None``: every point of ``x`` queries its own cloud
      (``offsets`` delimit the clouds; None = one cloud).  Returns
      (d2 [N][k], idx [N][k] global rows); gradients flow to ``x`` through
      both roles (query and neighbour).
    * ``queries`` with ``q_offsets``: cloud c's queries (rows
      [q_offsets[c], q_offsets[c+1]) of ``queries``) search cloud c of ``x``
      (``offsets``), all clouds in one persistent launch; idx are global
      rows of ``x``; gradients flow to both.
    * ``queries`` alone: k-NN of ``queries`` over all of ``x``.
    """
    if queries is not None and q_offsets is not None:
        if batch is None:
            if offsets is None:
                offsets = [0, x.shape[0]]
            batch = B.BatchKnn(offsets, x.shape[1], device=x.device)
        return _BatchQueryKnn.apply(queries, x, k, batch, q_offsets)
    if queries is not None:
        return _QueryKnn.apply(queries, x, k, leaf)
    if batch is None:
        if offsets is None:
            offsets = [0, x.shape[0]]
        batch = B.BatchKnn(offsets, x.shape[1], device=x.device)
    return _SelfKnn.apply(x, k, batch)
