"""``torch.autograd.Function`` around the tree evaluation and its adjoint walk.

Forward: build the tree over (x, v, m) and evaluate g, j, T at the active
rows (``ag_tree_build`` + ``ag_grav_eval``).  Backward: for the incoming
gradient w = dL/dg (read at the active rows), rebuild the tree from the saved
inputs (no interaction lists are kept from the forward pass) and run the
adjoint walk (``ag_tree_build`` + ``ag_grav_backward``), which returns
dL/dx and dL/dm for every particle.  Gradients flowing into the jerk or the
tidal tensor are not supported.  The adjoint is the tree approximation of the
exact gradient of the direct sum, not the derivative of the tree forward
(which is not smooth where a node's opening decision flips).
"""
from __future__ import annotations

import torch


class GravEval(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx, x, v, m, active_idx, theta, eps, G, n_leaf):
        n = x.shape[0]
        acc = torch.zeros((n, 3), dtype=torch.float64, device=x.device)
        jerk = torch.zeros((n, 3), dtype=torch.float64, device=x.device)
        tidal = torch.zeros((n, 6), dtype=torch.float64, device=x.device)
        ctx.tree_build(x, v, m, n_leaf)
        ctx.grav_eval(active_idx, theta, eps, G, acc, jerk, tidal)
        fctx.save_for_backward(x, v, m)
        fctx.ag = (ctx, active_idx, theta, eps, G, n_leaf)
        fctx.mark_non_differentiable(jerk, tidal)
        return acc, jerk, tidal

    @staticmethod
    def backward(fctx, g_acc, g_jerk, g_tidal):
        for g, name in ((g_jerk, "jerk"), (g_tidal, "tidal")):
            if g is not None and bool(torch.any(g != 0)):
                raise NotImplementedError(f"gradient through the {name} output is not supported")
        x, v, m = fctx.saved_tensors
        ctx, active_idx, theta, eps, G, n_leaf = fctx.ag
        n = x.shape[0]
        dldx = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        dldm = torch.empty((n,), dtype=torch.float64, device=x.device)
        if g_acc is None:
            return None, torch.zeros_like(x), None, torch.zeros_like(m), None, None, None, None, None
        w = g_acc.contiguous().to(torch.float64)
        ctx.tree_build(x, v, m, n_leaf)
        ctx.grav_backward(active_idx, w, theta, eps, G, dldx, dldm)
        return None, dldx, None, dldm, None, None, None, None, None


def grav_eval(ctx, x, v, m, active_idx=None, theta=0.6, eps=1e-3, G=1.0, n_leaf=16):
    """Differentiable tree gravity: returns (acc, jerk, tidal); acc carries
    gradients to x and m."""
    return GravEval.apply(ctx, x, v, m, active_idx, theta, eps, G, n_leaf)
