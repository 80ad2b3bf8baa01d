"""torch.autograd.Function around the HIP forward and adjoint kernels.

forward: Eq. 2 for every shot of the survey, storing checkpoints (or, with
the survey's full_history tune, the velocity of every step) in the survey's
own checkpoint workspace, which stays reserved for this call until its
backward has run or its graph is freed; a second forward issued while the
first still holds it gets a fresh allocation.
backward: grad_traces is dJ/dtraces for whatever loss the caller built (for
Eq. 1 it is the residual of Eq. 5); the adjoint kernels recompute each
checkpoint segment and correlate (Eq. 6-8); the finalize kernel returns
dJ/dlambda and dJ/dmu on the global model grid.  The illumination of the
same pass is left on the survey as ``last_illum`` for the preconditioner.
When rho requires grad the density correlation runs in the same adjoint pass
(joint inversion, an extension of the paper's fixed density); when the
wavelet requires grad the same pass records dJ/dwavelet (source-signature
estimation, also beyond the paper's known Ricker; not with rho at once).
"""
from __future__ import annotations

import weakref

import torch


class BoreholeFWI(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lam, mu, survey, rho, wavelet):
        ckpt, token = survey.checkout_ckpt()
        # the reservation ends with the backward, or with this context when no
        # backward ever runs (no_grad, a discarded graph)
        weakref.finalize(ctx, survey.release_ckpt, token)
        traces = survey.fwd_model(lam.detach(), mu.detach(), rho.detach(), wavelet,
                                  store_ckpt=True, ckpt=ckpt)
        ctx.survey = survey
        ctx.ckpt, ctx.token = ckpt, token
        ctx.save_for_backward(lam.detach(), mu.detach(), rho.detach(), wavelet)
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        lam, mu, rho, wavelet = ctx.saved_tensors
        survey = ctx.survey
        resid = grad_traces.contiguous().float()
        g_rho = g_wav = None
        if ctx.needs_input_grad[3] and ctx.needs_input_grad[4]:
            survey.release_ckpt(ctx.token)
            raise NotImplementedError("the density and wavelet gradients are not taken in one "
                                      "adjoint pass")
        if ctx.needs_input_grad[3]:
            acc, acc_rho = survey.adjoint_model_density(lam, mu, rho, wavelet, resid,
                                                        ckpt=ctx.ckpt)
            g_rho = survey.gradient_density(rho, acc_rho)
        elif ctx.needs_input_grad[4]:
            acc, g_wav = survey.adjoint_model_wavelet(lam, mu, rho, wavelet, resid,
                                                      ckpt=ctx.ckpt)
        else:
            acc = survey.adjoint_model(lam, mu, rho, wavelet, resid, ckpt=ctx.ckpt)
        g_lam, g_mu, illum = survey.gradient(mu, acc)
        survey.last_illum = illum
        ctx.ckpt = None
        survey.release_ckpt(ctx.token)
        return g_lam, g_mu, None, g_rho, g_wav


class Moduli(torch.autograd.Function):
    """Eq. 3-4 as a differentiable op (forward and chain rule in the library),
    so that BoreholeFWI gradients reach a (Vp, Vs) parameterisation."""

    @staticmethod
    def forward(ctx, vp, vs, rho):
        from ._lib import moduli
        lam, mu = moduli(vp.detach().contiguous(), vs.detach().contiguous(),
                         rho.detach().contiguous())
        ctx.save_for_backward(vp.detach(), vs.detach(), rho.detach())
        return lam, mu

    @staticmethod
    def backward(ctx, g_lam, g_mu):
        from ._lib import moduli_grad
        vp, vs, rho = ctx.saved_tensors
        if g_lam is None:
            g_lam = torch.zeros_like(vp)
        if g_mu is None:
            g_mu = torch.zeros_like(vp)
        if ctx.needs_input_grad[2]:
            g_vp, g_vs, g_rho = moduli_grad(vp, vs, rho, g_lam.contiguous(), g_mu.contiguous(),
                                            density=True)
            return g_vp, g_vs, g_rho
        g_vp, g_vs = moduli_grad(vp, vs, rho, g_lam.contiguous(), g_mu.contiguous())
        return g_vp, g_vs, None
