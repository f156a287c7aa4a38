"""torch.autograd.Function around ssoct_render / ssoct_backward.

Forward: the complex volume V(z, c, phi) of one sweep.  Backward: the
hand-written adjoint of the whole chain (ssoct_backward), which recomputes the
rescaled, chirped frames instead of storing any intermediate stack; only the
frames and the small parameter tensors are saved.
"""
from __future__ import annotations

import torch

from .api import Plan


class SsoctRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, frames, z, zernike, disp_phase, plan: Plan, lam, pitch):
        zf = float(z.detach().cpu())
        zc = zernike.detach().cpu().double().tolist() if zernike is not None else None
        ph = disp_phase.detach().cpu().double().tolist() if disp_phase is not None else None
        V = plan.render(frames, lam, pitch, zf, ph, zc)
        ctx.plan, ctx.lam, ctx.pitch = plan, lam, pitch
        ctx.params = (zf, zc, ph)
        ctx.has = (zernike is not None, disp_phase is not None)
        ctx.save_for_backward(frames, z)
        return V

    @staticmethod
    def backward(ctx, grad_v):
        frames, z = ctx.saved_tensors
        zf, zc, ph = ctx.params
        g = ctx.plan.backward(frames, ctx.lam, ctx.pitch, zf, grad_v.contiguous().to(torch.complex64), ph, zc)
        g = g.cpu()
        dz = g[1].to(z.dtype).reshape(z.shape)
        dc = g[2:17].clone() if ctx.has[0] else None
        dphi = g[17:].clone() if ctx.has[1] else None
        return None, dz, dc, dphi, None, None, None


def render(frames, z, zernike, disp_phase, plan: Plan, lam, pitch):
    """Differentiable render: V as a function of z (0-d tensor), zernike [15] and disp_phase [T]."""
    return SsoctRender.apply(frames, z, zernike, disp_phase, plan, lam, pitch)
