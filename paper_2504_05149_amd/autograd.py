"""Differentiable SE(2) convolution with a radial-profile kernel.

out = S_K[f, rho(prof)] on the grid, with rho the radial-profile kernel
P[l][j][i] = sum_q prof[q][l] H_q(x_ij) (raw samples, no renormalisation, so the
map prof -> P is linear).  Gradients (all computed by the HIP library):

* dL/df    = adjoint apply of dL/dout with the kernel table (correlation);
* sum_b dL/dP_b = Re iDFT(sum_b G_b^ . conj f_b^) with the fields' own FFC tables
             (se2conv_field_coeffs), accumulated spectrally (se2conv_kernel_grad);
* dL/dprof = hat-basis transpose of sum_b dL/dP_b (se2conv_profile_grad).

On FP32 plans with register kernels the backward is fused (se2conv_backward):
one y pass produces the adjoint product for dL/df and accumulates sum_b dL/dP_b
against the fields' packed spectra (se2conv_field_spectra / se2conv_apply_save).

checkpoint=True keeps the field tables (or spectra, saved by the forward's own y
pass) for the backward pass; checkpoint=False recomputes them in the backward pass.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .api import Plan, RadialProfile


class RadialProfileConv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, prof, plan: Plan, shape_idx: int, r_max: float, checkpoint: bool):
        f = f.detach().contiguous()
        prof = prof.detach().contiguous()
        table = plan.coeffs(shape_idx, [RadialProfile(prof, r_max, norm=L.KNORM_NONE)])
        ctx.fused = plan.fused_supported(shape_idx)
        ctx.ftabs = ctx.spectra = None
        if ctx.fused and checkpoint:
            out, ctx.spectra = plan.apply_save(shape_idx, f, table)
        else:
            out = plan.apply(shape_idx, f, table)
            if checkpoint:
                ctx.ftabs = plan.field_coeffs(shape_idx, f)
        ctx.plan, ctx.shape_idx, ctx.r_max = plan, shape_idx, r_max
        ctx.table = table
        ctx.n_knots = prof.shape[0]
        ctx.save_for_backward(f)
        return out

    @staticmethod
    def backward(ctx, g):
        (f,) = ctx.saved_tensors
        plan, sidx = ctx.plan, ctx.shape_idx
        g = g.contiguous()
        grad_f = grad_prof = None
        if ctx.fused:
            spectra = ctx.spectra if ctx.spectra is not None else plan.field_spectra(sidx, f)
            grad_f, grad_p = plan.backward(sidx, g, ctx.table, spectra)
            if ctx.needs_input_grad[1]:
                grad_prof = plan.profile_grad(sidx, grad_p, ctx.n_knots, ctx.r_max)
            return (grad_f if ctx.needs_input_grad[0] else None), grad_prof, None, None, None, None
        if ctx.needs_input_grad[0]:
            grad_f = plan.apply(sidx, g, ctx.table, adjoint=True)
        if ctx.needs_input_grad[1]:
            ftabs = ctx.ftabs if ctx.ftabs is not None else plan.field_coeffs(sidx, f)
            # sum_b dL/dP_b, accumulated in the spectral domain and inverted once
            grad_p = plan.kernel_grad(sidx, g, ftabs)
            grad_prof = plan.profile_grad(sidx, grad_p, ctx.n_knots, ctx.r_max)
        return grad_f, grad_prof, None, None, None, None


def radial_profile_conv(f: torch.Tensor, prof: torch.Tensor, plan: Plan, shape_idx: int = 0, r_max: float = 0.5,
                        checkpoint: bool = True) -> torch.Tensor:
    """f: [B, M, Ny, Nx] (plan dtype); prof: [n_knots, M] float64 on the same device."""
    return RadialProfileConv.apply(f, prof, plan, shape_idx, r_max, checkpoint)
