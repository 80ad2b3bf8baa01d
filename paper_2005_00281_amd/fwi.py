"""Gradient-descent FWI iteration (the five steps of the paper's workflow
figure: forward modelling, data residue, adjoint modelling, gradient,
model update), every step on the GPU through libbhfwi.

The model is carried as P and S velocities (density fixed, as the Method
section treats it); each iteration converts them to moduli (Eq. 3-4), runs for
each group of shots the forward with checkpoints (Eq. 2), the misfit (Eq. 1,
5), the adjoint with the fused correlation (Eq. 6-8) and the gradient
finalize (summed over groups), then the diagonal preconditioner, the update
(Eq. 9-10) and the conversion back (Eq. 11-12).  All buffers persist across
iterations so that the captured HIP graphs replay; the groups share one set
of workspaces.

With line_search=True the step length comes from a parabolic line search:
a trial update with the greatest-change rule, one forward pass (no
checkpoints) of every group on the trial model for its misfit, and the
minimum of the parabola through the two misfits and the slope along the
preconditioned gradient (bhfwi_line_search); the whole iteration stays on
the device without a host synchronisation.

With autograd=True the gradient of each group comes from the
torch.autograd.Function around the forward and adjoint kernels
(BoreholeFWI): the traces are its output, the misfit of Eq. 1 is a torch
expression of them (summed in float64), and loss.backward() runs the
checkpoint recompute, the adjoint with the fused correlation and the
finalize; the illumination of the same pass feeds the preconditioner.  The
kernels and workspaces are the same as on the direct path.

Extensions beyond the paper's fixed density and illumination preconditioner
(all optional, off by default):
  density=True     joint inversion: the adjoint pass also accumulates
                   dJ/drho, preconditioned with the illumination and stepped
                   with its own greatest-change rule (eta_rho, rho_bounds)
                   before the moduli update;
  precond="pseudo_hessian"
                   the virtual-source pseudo-Hessian diagonals H_lambda and
                   H_mu of the same adjoint pass replace the illumination as
                   the diagonals of the lambda and mu preconditioners;
  row_weight       a weight per radial row of the model (radial_taper) applied
                   on top of the diagonal, muting the near-wall gradient.
"""
from __future__ import annotations

import torch

from . import _lib


class Inversion:
    def __init__(self, surveys, vp, vs, rho, wavelets, observed, mask, eps=1e-3, eta=0.02,
                 bounds=(1000.0, 7000.0, 300.0, 4500.0), line_search=False, density=False,
                 eta_rho=None, rho_bounds=(1000.0, 3500.0), precond="illum", row_weight=None,
                 autograd=False):
        if precond not in ("illum", "pseudo_hessian"):
            raise ValueError("precond must be 'illum' or 'pseudo_hessian'")
        if autograd and precond != "illum":
            raise ValueError("the autograd path returns the illumination as its only "
                             "preconditioner diagonal")
        self.autograd = bool(autograd)
        if density and line_search:
            raise ValueError("the line search steps lambda and mu only; use density without it")
        if not isinstance(surveys, (list, tuple)):
            surveys, wavelets, observed = [surveys], [wavelets], [observed]
        self.surveys = list(surveys)
        self.vp, self.vs, self.rho = vp, vs, rho
        self.wavelets, self.observed = list(wavelets), list(observed)
        self.mask = mask
        self.eps, self.eta, self.bounds = float(eps), float(eta), tuple(bounds)
        dev = vp.device
        need = {k: max(getattr(sv.sizes, k + "_bytes") for sv in self.surveys)
                for k in ("fwd_ws", "ckpt", "adj_ws")}
        self.pool = {"fwd": torch.empty(max(1, need["fwd_ws"]), dtype=torch.uint8, device=dev),
                     "ckpt": torch.empty(max(1, need["ckpt"]), dtype=torch.uint8, device=dev),
                     "adj": torch.empty(max(1, need["adj_ws"]), dtype=torch.uint8, device=dev)}
        for sv in self.surveys:
            sv.use_workspaces(self.pool)
        # the autograd path's backward allocates its own accumulators
        self.acc = (None if self.autograd else
                    torch.empty(max(sv.sizes.acc_elems for sv in self.surveys),
                                dtype=torch.float32, device=dev))
        self.traces = [torch.empty(sv.sizes.trace_elems, dtype=torch.float32, device=dev)
                       for sv in self.surveys]
        self.resid = [torch.empty_like(t) for t in self.traces]
        self.lam = torch.empty_like(vp)
        self.mu = torch.empty_like(vp)
        self.g_lam = torch.empty_like(vp)
        self.g_mu = torch.empty_like(vp)
        self.illum = torch.empty_like(vp)
        self.J = torch.zeros((), dtype=torch.float64, device=dev)
        self.density = bool(density)
        self.hessian = precond == "pseudo_hessian"
        self.eta_rho = float(eta if eta_rho is None else eta_rho)
        self.rho_bounds = tuple(rho_bounds)
        self.row_weight = row_weight
        cells = max(sv.sizes.cells for sv in self.surveys)
        if self.density:
            self.acc_rho = torch.empty(2 * cells, dtype=torch.float32, device=dev)
            self.g_rho = torch.empty_like(vp)
            self.alpha_rho = torch.zeros((), dtype=torch.float32, device=dev)
        if self.hessian:
            self.acc_h = torch.empty(2 * cells, dtype=torch.float32, device=dev)
            self.h_lam = torch.empty_like(vp)
            self.h_mu = torch.empty_like(vp)
        self.line_search = bool(line_search)
        self.after_group = None  # optional callback(stage, group) after each group's work
        if self.line_search:
            self.J1 = torch.zeros((), dtype=torch.float64, device=dev)
            self.gpg = torch.zeros((), dtype=torch.float64, device=dev)
            self.lam1 = torch.empty_like(vp)
            self.mu1 = torch.empty_like(vp)

    def gradient(self):
        """Eq. 2, 1, 5, 6-8 and the finalize over every group; leaves the
        misfit in self.J and the raw gradient and illumination on the model."""
        if self.autograd:
            return self._gradient_autograd()
        _lib.moduli(self.vp, self.vs, self.rho, out=(self.lam, self.mu))
        for g, sv in enumerate(self.surveys):
            ckpt = self.pool["ckpt"]
            sv.fwd_model(self.lam, self.mu, self.rho, self.wavelets[g], store_ckpt=True,
                         ckpt=ckpt, traces=self.traces[g])
            sv.misfit(self.traces[g], self.observed[g], resid=self.resid[g], J=self.J,
                      accumulate=g > 0)
            if self.density or self.hessian:
                sv.adjoint_model_ex(self.lam, self.mu, self.rho, self.wavelets[g],
                                    self.resid[g], ckpt=ckpt, acc=self.acc,
                                    density=self.density, hessian=self.hessian,
                                    acc_rho=self.acc_rho if self.density else None,
                                    acc_h=self.acc_h if self.hessian else None)
                if self.density:
                    sv.gradient_density(self.rho, self.acc_rho, out=self.g_rho,
                                        accumulate=g > 0)
                if self.hessian:
                    sv.gradient_hessian(self.acc_h, out=(self.h_lam, self.h_mu),
                                        accumulate=g > 0)
            else:
                sv.adjoint_model(self.lam, self.mu, self.rho, self.wavelets[g], self.resid[g],
                                 ckpt=ckpt, acc=self.acc)
            sv.gradient(self.mu, self.acc, out=(self.g_lam, self.g_mu, self.illum),
                        accumulate=g > 0)
            if self.after_group:
                self.after_group("gradient", g)
        return self.J

    def _gradient_autograd(self):
        """gradient() through BoreholeFWI and loss.backward()."""
        from .autograd import BoreholeFWI
        _lib.moduli(self.vp, self.vs, self.rho, out=(self.lam, self.mu))
        lam = self.lam.detach().requires_grad_(True)
        mu = self.mu.detach().requires_grad_(True)
        rho = self.rho.detach().requires_grad_(self.density)
        for g, sv in enumerate(self.surveys):
            traces = BoreholeFWI.apply(lam, mu, sv, rho, self.wavelets[g])
            r = (traces - self.observed[g]).double()
            loss = 0.5 * torch.dot(r, r)
            loss.backward()
            if g == 0:
                self.J.copy_(loss.detach())
                self.illum.copy_(sv.last_illum)
            else:
                self.J.add_(loss.detach())
                self.illum.add_(sv.last_illum)
            sv.last_illum = None
            if self.after_group:
                self.after_group("gradient", g)
        self.g_lam.copy_(lam.grad)
        self.g_mu.copy_(mu.grad)
        if self.density:
            self.g_rho.copy_(rho.grad)
        return self.J

    def iterate(self):
        """One iteration; returns (J, alpha) as device scalars (no host sync).
        J is a copy: the misfit buffer is overwritten by the next iteration."""
        self.gradient()
        sv = self.surveys[0]
        if self.density:
            sv.precondition_diag(self.g_rho, self.mask, self.eps, self.illum, self.row_weight)
            sv.update_density(self.rho, self.g_rho, self.mask, self.eta_rho, *self.rho_bounds,
                              alpha=self.alpha_rho)
        if not self.line_search:
            self._precondition()
            alpha = sv.update(self.lam, self.mu, self.rho, self.g_lam, self.g_mu, self.mask,
                              self.eta, bounds=self.bounds)
        else:
            alpha = self._line_search_step()
        _lib.velocities(self.lam, self.mu, self.rho, out=(self.vp, self.vs))
        return self.J.clone(), alpha

    def _precondition(self, gpg=None):
        """The lambda and mu gradients through the chosen diagonal (and the
        row weights); gpg (nullable) receives sum g . P g over both."""
        sv = self.surveys[0]
        if not self.hessian and self.row_weight is None:
            sv.precondition(self.illum, self.mask, self.eps, self.g_lam, self.g_mu, gpg=gpg)
            return
        d_l, d_m = (self.h_lam, self.h_mu) if self.hessian else (self.illum, self.illum)
        sv.precondition_diag(self.g_lam, self.mask, self.eps, d_l, self.row_weight, gpg=gpg)
        sv.precondition_diag(self.g_mu, self.mask, self.eps, d_m, self.row_weight, gpg=gpg,
                             accumulate=True)

    def _line_search_step(self):
        sv = self.surveys[0]
        self._precondition(gpg=self.gpg)
        self.lam1.copy_(self.lam)
        self.mu1.copy_(self.mu)
        alpha1 = sv.update(self.lam1, self.mu1, self.rho, self.g_lam, self.g_mu, self.mask,
                           self.eta, bounds=self.bounds)
        for g, svg in enumerate(self.surveys):
            svg.fwd_model(self.lam1, self.mu1, self.rho, self.wavelets[g],
                          traces=self.traces[g])
            svg.misfit(self.traces[g], self.observed[g], resid=self.resid[g], J=self.J1,
                       accumulate=g > 0)
            if self.after_group:
                self.after_group("line search", g)
        alpha = sv.line_search(self.J, self.J1, self.gpg, alpha1)
        sv.update(self.lam, self.mu, self.rho, self.g_lam, self.g_mu, self.mask, self.eta,
                  bounds=self.bounds, alpha_in=alpha)
        return alpha
