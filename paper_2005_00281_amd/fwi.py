"""Gradient-descent FWI iteration (the five steps of the paper's workflow
figure: forward modelling, data residue, adjoint modelling, gradient,
model update), every step on the GPU through libbhfwi.

The model is carried as P and S velocities (density fixed, as the Method
section treats it); each iteration converts them to moduli (Eq. 3-4), runs the
forward with checkpoints (Eq. 2), the misfit (Eq. 1, 5), the adjoint with the
fused correlation (Eq. 6-8), the gradient finalize, the diagonal
preconditioner, the update (Eq. 9-10) and the conversion back (Eq. 11-12).
All buffers persist across iterations so that the captured HIP graphs replay.
"""
from __future__ import annotations

import torch

from . import _lib


class Inversion:
    def __init__(self, survey, vp, vs, rho, wavelet, observed, mask, eps=1e-3, eta=0.02,
                 bounds=(1000.0, 7000.0, 300.0, 4500.0)):
        self.sv = survey
        self.vp, self.vs, self.rho = vp, vs, rho
        self.wavelet, self.observed = wavelet, observed
        self.mask = mask
        self.eps, self.eta, self.bounds = float(eps), float(eta), tuple(bounds)
        z = survey.sizes
        dev = vp.device
        self.lam = torch.empty_like(vp)
        self.mu = torch.empty_like(vp)
        self.traces = torch.empty(z.trace_elems, dtype=torch.float32, device=dev)
        self.resid = torch.empty(z.trace_elems, dtype=torch.float32, device=dev)
        self.acc = torch.empty(z.acc_elems, dtype=torch.float32, device=dev)
        self.g_lam = torch.empty_like(vp)
        self.g_mu = torch.empty_like(vp)
        self.illum = torch.empty_like(vp)
        self.ckpt = survey.workspace("ckpt")

    def iterate(self):
        """One iteration; returns (J, alpha) as device scalars (no host sync)."""
        sv = self.sv
        _lib.moduli(self.vp, self.vs, self.rho, out=(self.lam, self.mu))
        sv.fwd_model(self.lam, self.mu, self.rho, self.wavelet, store_ckpt=True,
                     ckpt=self.ckpt, traces=self.traces)
        _, J = sv.misfit(self.traces, self.observed, resid=self.resid)
        sv.adjoint_model(self.lam, self.mu, self.rho, self.wavelet, self.resid, ckpt=self.ckpt,
                         acc=self.acc)
        sv.gradient(self.mu, self.acc, out=(self.g_lam, self.g_mu, self.illum))
        sv.precondition(self.illum, self.mask, self.eps, self.g_lam, self.g_mu)
        alpha = sv.update(self.lam, self.mu, self.rho, self.g_lam, self.g_mu, self.mask, self.eta,
                          bounds=self.bounds)
        _lib.velocities(self.lam, self.mu, self.rho, out=(self.vp, self.vs))
        return J, alpha
