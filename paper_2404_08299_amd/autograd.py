"""PageRank as a differentiable torch operation.

The forward pass is the weighted PageRank fixed point
    r = alpha * A r + (1 - alpha) s,   A[v][u] = P_uv (one entry per edge u -> v),
solved by pr_weighted; the backward pass solves the adjoint fixed point
    lambda = g + alpha * A^T lambda
with pr_adjoint and returns dL/dP_uv = alpha * r_u * lambda_v and
dL/ds = (1 - alpha) * lambda. Both run in the HIP library; ranks stay FP64.

The weights P are used as given. A normalisation of raw weights (for example
P_uv = w_uv / sum_v w_uv) belongs outside this Function, in torch, so that
autograd chains through it.
"""
from __future__ import annotations

import torch

from . import prhip


class PageRankFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, weights, teleport, graph, alpha=prhip.ALPHA, tol=prhip.TOL,
                max_iter=prhip.MAX_ITERATIONS, adjoint_tol=None):
        weights = weights.contiguous()
        tele = teleport.contiguous() if teleport is not None else None
        res = prhip.weighted(graph, weights, tele, alpha=alpha, tol=tol, max_iter=max_iter)
        r = res.ranks
        ctx.save_for_backward(weights, r)
        ctx.graph = graph
        ctx.alpha = alpha
        ctx.tol = tol if adjoint_tol is None else adjoint_tol
        ctx.max_iter = max_iter
        ctx.has_teleport = teleport is not None
        return r

    @staticmethod
    def backward(ctx, grad_r):
        weights, r = ctx.saved_tensors
        need_w = ctx.needs_input_grad[0]
        need_s = ctx.needs_input_grad[1] and ctx.has_teleport
        if not (need_w or need_s):
            return None, None, None, None, None, None, None
        gw, gs, _ = prhip.adjoint(ctx.graph, weights, r, grad_r.contiguous().to(torch.float64),
                                  alpha=ctx.alpha, tol=ctx.tol, max_iter=ctx.max_iter,
                                  want_weights=need_w, want_teleport=need_s)
        return gw, gs, None, None, None, None, None


def pagerank(weights, teleport, graph, alpha=prhip.ALPHA, tol=prhip.TOL,
             max_iter=prhip.MAX_ITERATIONS, adjoint_tol=None):
    """r = PageRank(P, s) on `graph` (a prhip.DeviceGraph); differentiable in
    `weights` (P in in-CSR order) and `teleport` (s, or None for 1/n)."""
    return PageRankFn.apply(weights, teleport, graph, alpha, tol, max_iter, adjoint_tol)
