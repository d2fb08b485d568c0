"""torch.autograd.Function wrappers around libgsr's forward and hand-written
backward (Sec. 3.3: every gradient of the rasterizer is computed explicitly).

GaussRender's backward is the library's adjoint (gsr_render_bwd): it
recomputes transmittance back to front from the forward's per-pixel state
(final transmittance and last composited position) instead of storing
per-pair values, and returns gradients for the activated Gaussian parameters
and the camera pose (Sec. 3.3 and Sec. 3.4). L1Loss and TrackLoss put the
library's loss kernels (Eq. 9 / the L1 part of Eq. 10, and Eq. 15) behind
autograd, so a mapping or tracking step can be written as loss.backward()
followed by a torch optimiser.
"""
from __future__ import annotations

import torch

from . import gsr

_PARAMS = ("means", "scales", "quats", "opacities", "colors")


class GaussRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacities, colors, pose7, camera, opts):
        color, depth, alpha, state = gsr.render_fwd(means, scales, quats, opacities, colors, pose7, camera, opts)
        # saved so that autograd rejects a backward after an in-place change of
        # any of them (the library's backward re-reads these buffers)
        ctx.save_for_backward(means, scales, quats, opacities, colors, pose7)
        ctx.state = state
        return color, depth, alpha

    @staticmethod
    def backward(ctx, gC, gD, gA):
        means = ctx.saved_tensors[0]  # unpacking runs autograd's version check
        state = ctx.state
        if state is None:
            raise RuntimeError("GaussRender: the backward of one forward can run only once")
        H, W = state.shape
        if gC is None:
            gC = torch.zeros((3, H, W), device=means.device, dtype=torch.float32)
        if gD is None:
            gD = torch.zeros((H, W), device=means.device, dtype=torch.float32)
        need = ctx.needs_input_grad
        out = gsr.render_bwd(state, gC, gD, gA, want_params=any(need[:5]), want_pose=need[5])
        state.release()
        ctx.state = None
        grads = [out[k] if need[i] else None for i, k in enumerate(_PARAMS)]
        grads.append(out["pose7"] if need[5] else None)
        return (*grads, None, None)


def render(means, scales, quats, opacities, colors, pose7, camera: gsr.Camera, opts: gsr.RasterOpts | None = None):
    """Differentiable render -> (color [3,H,W], depth [H,W], alpha [H,W])."""
    return GaussRender.apply(means, scales, quats, opacities, colors, pose7, camera, opts or gsr.RasterOpts())


class L1Loss(torch.autograd.Function):
    """Mapping L1 (Eq. 9 and the L1 part of Eq. 10): w_c mean|C - C*| + w_d mean|D - D*|."""

    @staticmethod
    def forward(ctx, color, depth, tgt_color, tgt_depth, w_color, w_depth):
        loss, gC, gD = gsr.loss_l1(color, depth, tgt_color, tgt_depth, w_color, w_depth)
        ctx.save_for_backward(gC, gD)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        gC, gD = ctx.saved_tensors
        return gC * g, gD * g, None, None, None, None


def loss_l1(color, depth, tgt_color, tgt_depth, w_color=1.0, w_depth=1.0):
    return L1Loss.apply(color.contiguous(), depth.contiguous(), tgt_color, tgt_depth, float(w_color), float(w_depth))


class TrackLoss(torch.autograd.Function):
    """Eq. 15 with the supplement's inlier and alpha^3 masks; the masks are
    constants, so no gradient reaches alpha."""

    @staticmethod
    def forward(ctx, color, depth, alpha, obs_color, obs_depth, lambda_c, inlier_mult):
        loss, gC, gD, _ = gsr.loss_track(color, depth, alpha, obs_color, obs_depth, lambda_c, inlier_mult)
        ctx.save_for_backward(gC, gD)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        gC, gD = ctx.saved_tensors
        return gC * g, gD * g, None, None, None, None, None


def loss_track(color, depth, alpha, obs_color, obs_depth, lambda_c=0.5, inlier_mult=50.0):
    return TrackLoss.apply(color.contiguous(), depth.contiguous(), alpha.contiguous(), obs_color, obs_depth,
                           float(lambda_c), float(inlier_mult))
