"""torch.autograd.Function around libgsr's forward and hand-written backward.

The backward is the library's adjoint (gsr_render_bwd): it recomputes
transmittance back to front from the forward's saved per-pixel state instead
of storing per-pair values, and returns gradients for the activated Gaussian
parameters and the camera pose (Sec. 3.3 and Sec. 3.4 of the paper).
"""
from __future__ import annotations

import torch

from . import gsr


class GaussRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacities, colors, pose7, camera, opts):
        color, depth, alpha, state = gsr.render_fwd(means, scales, quats, opacities, colors, pose7, camera, opts)
        ctx.state = state
        return color, depth, alpha

    @staticmethod
    def backward(ctx, gC, gD, gA):
        state = ctx.state
        means = state.keep[0]
        H, W = gsr_shape(state)
        if gC is None:
            gC = torch.zeros((3, H, W), device=means.device, dtype=torch.float32)
        if gD is None:
            gD = torch.zeros((H, W), device=means.device, dtype=torch.float32)
        need = ctx.needs_input_grad
        out = gsr.render_bwd(state, gC, gD, gA, want_params=any(need[:5]), want_pose=need[5])
        state.release()
        ctx.state = None
        names = ("means", "scales", "quats", "opacities", "colors")
        grads = [out[k] if need[i] else None for i, k in enumerate(names)]
        grads.append(out["pose7"] if need[5] else None)
        return (*grads, None, None)


def gsr_shape(state) -> tuple[int, int]:
    return state.shape


def render(means, scales, quats, opacities, colors, pose7, camera: gsr.Camera, opts: gsr.RasterOpts | None = None):
    """Differentiable render -> (color [3,H,W], depth [H,W], alpha [H,W])."""
    return GaussRender.apply(means, scales, quats, opacities, colors, pose7, camera, opts or gsr.RasterOpts())
