"""torch.autograd.Function wrappers over the library's hand-written adjoints.

LogLik:       params [G, 6] -> log L [G] (eq. likelihood-pixels); backward
              multiplies the incoming gradient into d log L / d params, which
              the same library call returns (the k-space adjoint).
ShearLogPost: points [P, 5] = (g1, g2, mu_ln_s, sigma_ln_s, sigma_e) -> ln P [P]
              (eq. likelihood-shear); backward uses the softmax-weighted
              closed-form derivative of the log importance weights.
Both run entirely in the HIP library; the wrappers only route tensors.
"""
from __future__ import annotations

import torch

from . import api


class LogLik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, data, batch, method=0):
        ll, grad, status = api.loglik_grad(batch, data, params.detach(), method)
        ctx.save_for_backward(grad)
        ctx.mark_non_differentiable(status)
        return ll, status

    @staticmethod
    def backward(ctx, g_ll, g_status):
        (grad,) = ctx.saved_tensors
        return (g_ll.to(grad.dtype)[:, None] * grad, None, None, None)


def loglik(params, data, batch, method=0):
    """log L [G] (float64) with autograd support through the library adjoint."""
    ll, _ = LogLik.apply(params, data, batch, method)
    return ll


class ShearLogPost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pts, e1p, e2p, log10s, log10f, true_prior, interim=None):
        lp, grad = api.shear_posterior(e1p, e2p, log10s, log10f, pts.detach().double().contiguous(),
                                       true_prior, interim, want_grad=True)
        ctx.save_for_backward(grad)
        return lp

    @staticmethod
    def backward(ctx, g_lp):
        (grad,) = ctx.saved_tensors
        return (g_lp[:, None] * grad, None, None, None, None, None, None)


def shear_logpost(pts, e1p, e2p, log10s, log10f, true_prior, interim=None):
    """ln P(g, alpha | d) + const at points [P, 5] with autograd support."""
    return ShearLogPost.apply(pts, e1p, e2p, log10s, log10f, true_prior, interim)
