"""torch.autograd.Function wrappers around the library's edge-weight
derivative kernels (the differentiable pieces behind the constrained-SGD
edge scaling of Sec. 3.3.4, Alg. 1).

SmoothedVectors(w_E, X0, g, edges, colours, n_colours, sweeps) -> X_S
    the multicolour Gauss-Seidel smoothing of X0 (Sec. 3.2.1) on graph g with
    edge weights w_E (float32, one per undirected edge); backward runs the
    library's reverse colour steps (gradients for w_E and X0).

RayleighQuotients(w_E, U, edges, mode) -> R[m]
    R_i = u_i^T L(w) u_i / u_i^T B u_i on edge weights w_E (float64, one per
    undirected edge).  backward gives dR/dw_E by the library's FP64 kernel;
    U is held fixed (the quotient is stationary at eigenvectors).
"""
from __future__ import annotations

import torch

from . import graphreduce as G


class RayleighQuotients(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w_E, U, edges, mode=G.GR_RQ_IDENTITY):
        w_E = w_E.detach().contiguous()
        U = U.detach().contiguous()
        R, den = G.gr_rq_forward(edges, w_E, U, mode)
        ctx.save_for_backward(U, R, den)
        ctx.edges = edges
        ctx.mode = mode
        return R

    @staticmethod
    def backward(ctx, gR):
        U, R, den = ctx.saved_tensors
        gw = G.gr_rq_backward(ctx.edges, U, R, den, gR, ctx.mode)
        return gw, None, None, None


def rayleigh_quotients(w_E, U, edges, mode=G.GR_RQ_IDENTITY):
    return RayleighQuotients.apply(w_E, U, edges, mode)


class SmoothedVectors(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w_E, X0, g, edges, colours, n_colours, sweeps,
                store_states=False):
        w = G.gr_expand_edge_weights(edges, w_E.detach())
        gw_graph = G.DeviceGraph(g.row_ptr, g.col, w)
        X = X0.detach().contiguous().clone()
        G.gr_smooth(gw_graph, colours, n_colours, X, sweeps)
        ctx.save_for_backward(X0.detach().contiguous())
        ctx.graph = gw_graph
        ctx.edges = edges
        ctx.colours = colours
        ctx.n_colours = n_colours
        ctx.sweeps = sweeps
        ctx.store = store_states
        return X

    @staticmethod
    def backward(ctx, gX):
        (X0,) = ctx.saved_tensors
        gw, gX0 = G.gr_smooth_vjp(ctx.graph, ctx.edges, ctx.colours,
                                  ctx.n_colours, X0,
                                  gX.contiguous().to(torch.float32),
                                  ctx.sweeps, ctx.store)
        return gw, gX0.to(X0.dtype), None, None, None, None, None, None


def smoothed_vectors(w_E, X0, g, edges, colours, n_colours, sweeps,
                     store_states=False):
    return SmoothedVectors.apply(w_E, X0, g, edges, colours, n_colours,
                                 sweeps, store_states)
