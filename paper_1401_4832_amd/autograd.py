"""torch.autograd.Function over (h, J) for the per-site objectives.

forward: f_r = B_eff * g_r^reg for every site r (eq. g_regdef2 times B_eff),
evaluated by the library's forward kernel only.  backward: the gradient
(eqs. g_gradh2, g_gradJ2) is recomputed by the library -- energies, softmax
and residuals are evaluated again rather than kept from the forward pass (they
are B*N*q values, 2.1 GB at N = 500, B = 50000) -- and the upstream gradient
enters as a per-site multiplier applied inside the library.
"""
from __future__ import annotations

import torch

from . import api


class PLMObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, J, msa, w, beff, lambda_h=0.01, lambda_J=0.01):
        f, _, _ = api.objgrad(msa, w, beff, h.detach(), J.detach(), lambda_h, lambda_J, grad=False)
        ctx.save_for_backward(h, J, msa, w, beff)
        ctx.lam = (lambda_h, lambda_J)
        return f

    @staticmethod
    def backward(ctx, grad_f):
        h, J, msa, w, beff = ctx.saved_tensors
        scale = grad_f.detach().to(torch.float64).contiguous()
        _, gh, gJ = api.objgrad(msa, w, beff, h.detach(), J.detach(), *ctx.lam, grad=True,
                                grad_scale=scale)
        return gh, gJ, None, None, None, None, None


def plm_objective(h, J, msa, w, beff, lambda_h=0.01, lambda_J=0.01):
    """Per-site objectives f [N] (float64), differentiable in h [N, q] and J [N, N, q, q]."""
    return PLMObjective.apply(h, J, msa, w, beff, lambda_h, lambda_J)
