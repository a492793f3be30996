"""Batches of parameter draws and the chi^2 log-likelihood as a
torch.autograd.Function whose backward is libjt's hand-written adjoint.

Parameter layout per draw (the macro row): SIE (theta_E, q, phi, cx, cy) --
or, with main = "epl", EPL (theta_E, gamma, q, phi, cx, cy) -- then shear
(gamma1, gamma2), then (amp, R_sersic, n_sersic, q, phi, cx, cy) for each
source and then each lens-light component.  Subhalos: x, y, Rs and alpha_Rs
as [B, n] tensors (and r_trunc for truncated ones); gradients flow to x, y and
alpha_Rs.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Any, Optional

import numpy as np


@dataclass
class DrawBatch:
    macro: Any                      # [B, P] float64 (host)
    n_src: int
    n_ll: int = 0
    sub_x: Optional[Any] = None     # [B, n] float32 (device tensor or array)
    sub_y: Optional[Any] = None
    sub_Rs: Optional[Any] = None
    sub_alpha_Rs: Optional[Any] = None
    main: str = "sie"               # "sie" or "epl": the main deflector of the macro rows
    sub_r_trunc: Optional[Any] = None   # [B, n]: truncated (TNFW) subhalos


def macro_row(lens, source, lens_light=()):
    """The macro row of one scene (same order as the adjoint's gradient): an
    EPL main deflector when the lens has one, else its SIE."""
    if getattr(lens, "epl", None) is not None:
        e = lens.epl
        v = [e.theta_E, e.gamma, e.q, e.phi, e.cx, e.cy]
    else:
        v = [lens.sie.theta_E, lens.sie.q, lens.sie.phi, lens.sie.cx, lens.sie.cy]
    v += [lens.shear.gamma1, lens.shear.gamma2]
    for c in list(source) + list(lens_light):
        v += [c.amp, c.R_sersic, c.n_sersic, c.q, c.phi, c.cx, c.cy]
    return np.array(v, dtype=np.float64)


def _make_function():
    import torch

    class Chi2LogLikelihood(torch.autograd.Function):
        """log L(macro, sub_x, sub_y, sub_alpha_Rs) per draw.  forward runs the
        batched forward model only; backward runs the adjoint, which recomputes
        the traced positions instead of keeping them from the forward."""

        @staticmethod
        def forward(fctx, macro, sub_x, sub_y, sub_alpha, jt, grid, n_src, n_ll, sub_Rs, psf, data, inv_var):
            batch = DrawBatch(macro.detach().cpu().numpy(), n_src, n_ll, sub_x.detach(), sub_y.detach(),
                              sub_Rs, sub_alpha.detach())
            logL = jt.chi2(grid, batch, data, inv_var, psf)
            fctx.save_for_backward(macro, sub_x, sub_y, sub_alpha)
            fctx.args = (jt, grid, n_src, n_ll, sub_Rs, psf, data, inv_var)
            return logL

        @staticmethod
        def backward(fctx, grad_out):
            macro, sub_x, sub_y, sub_alpha = fctx.saved_tensors
            jt, grid, n_src, n_ll, sub_Rs, psf, data, inv_var = fctx.args
            batch = DrawBatch(macro.detach().cpu().numpy(), n_src, n_ll, sub_x.detach(), sub_y.detach(), sub_Rs,
                              sub_alpha.detach())
            _, gm, gs = jt.chi2_grad(grid, batch, data, inv_var, psf)
            go = grad_out.to(gm.device, torch.float32)
            g_macro = (gm * go[:, None]).to(macro.device, macro.dtype)
            gsub = gs * go[:, None, None]
            return (g_macro, gsub[..., 0].to(sub_x.dtype), gsub[..., 1].to(sub_y.dtype),
                    gsub[..., 2].to(sub_alpha.dtype), None, None, None, None, None, None, None, None)

    return Chi2LogLikelihood


_FN = None


def chi2_loglike(jt, grid, macro, sub_x, sub_y, sub_Rs, sub_alpha, n_src, n_ll, data, inv_var, psf=None):
    """Differentiable log L per draw (float64 [B]) on libjt's kernels."""
    global _FN
    if _FN is None:
        _FN = _make_function()
    return _FN.apply(macro, sub_x, sub_y, sub_alpha, jt, grid, n_src, n_ll, sub_Rs, psf, data, inv_var)
