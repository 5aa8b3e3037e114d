"""torch.autograd.Function over the library's loss and its hand-written adjoints.

    loss = sum_d || rho_c(z) q_d - x_d ||^2          (eq. "nnls")

with rho_c(z) the route-choice parameterisation of the assignment matrix
(eqs. "logit", "flow", "assign": softmax of per-path logits z within each OD,
times the per-path lag ratios).  Forward and backward run in libdode's kernels;
the residual is recomputed in backward rather than stored.
"""
from __future__ import annotations

import torch

from . import _lib


class DodeLoss(torch.autograd.Function):
    """DodeLoss.apply(Q, z, dar, cluster, routes, Rr, X) -> scalar loss (FP64 tensor).

    Q   [n][T][P] demand of n days of `cluster` (state dtype of `dar`)
    z   [n_paths] route logits (float32 or float64)
    Rr  [K][T][n_pairs] per-pair lag ratios (dtype of z)
    X   [n][H][L] observations
    The values rho_c(z) are installed in `dar` (dar_set_values) by the forward
    and installed again from the saved z by the backward, so several forwards
    with different logits on one `dar` (a sum of losses, a line search) each
    get the gradient of their own rho_c(z).  After a backward, `dar` holds the
    values of that call's z.
    """

    @staticmethod
    def _install(dar, cluster, routes, Rr, z):
        P, L, T, H, K = dar.dims
        W = torch.empty((K, T, routes.nnz), dtype=z.dtype, device=z.device)
        _lib.dar_from_logits(routes, Rr, z, W)
        Wd = W if W.dtype == dar.state_dtype else W.to(dar.state_dtype)
        _lib.dar_set_values(dar, cluster, Wd.contiguous())

    @staticmethod
    def forward(ctx, Q, z, dar, cluster, routes, Rr, X):
        DodeLoss._install(dar, cluster, routes, Rr, z)
        loss = torch.empty(Q.shape[0], dtype=torch.float64, device=Q.device)
        _lib.dode_loss(dar, cluster, Q, X, loss)
        ctx.dar, ctx.cluster, ctx.routes = dar, cluster, routes
        ctx.save_for_backward(Q, z, Rr, X)
        return loss.sum()

    @staticmethod
    def backward(ctx, g):
        Q, z, Rr, X = ctx.saved_tensors
        dar, routes = ctx.dar, ctx.routes
        P, L, T, H, K = dar.dims
        go = float(g)
        # the residual is recomputed with rho_c of this call's logits
        DodeLoss._install(dar, ctx.cluster, routes, Rr, z)
        dQ = torch.empty_like(Q) if ctx.needs_input_grad[0] else None
        dz = None
        dW = None
        if ctx.needs_input_grad[1]:
            dW = torch.empty((K, T, routes.nnz), dtype=dar.state_dtype, device=Q.device)
        _lib.dode_loss_bwd(dar, ctx.cluster, Q, X, go, dQ=dQ, dW=dW)
        if dW is not None:
            dz = torch.empty_like(z)
            _lib.dar_logits_bwd(routes, Rr, z, dW.to(z.dtype).contiguous(), dz)
        return dQ, dz, None, None, None, None, None


def dode_loss(Q, z, dar, cluster, routes, Rr, X):
    return DodeLoss.apply(Q, z, dar, cluster, routes, Rr, X)
