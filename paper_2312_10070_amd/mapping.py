"""Global-map post-processing (supplement, further implementation details):
after the saved sub-maps are merged into one global map (gsr.merge_submap:
a Gaussian joins if the map so far has no mean within rho), the global map's
colours are refined. Reading taken: refinement is Adam on the RGB colours
only (Sec. 3.2 optimises RGB directly), minimising the colour loss of Eq. 10,
(1 - lambda) L1 + lambda (1 - SSIM), against the keyframes taken in turn, one
per iteration; means, scales, rotations and opacities stay fixed. Every step
is a library call (forward render, loss kernels, hand-written backward of
the colours only, Adam)."""
from __future__ import annotations

import torch

from . import gsr


def refine_colors(params: dict, frames: list, camera: gsr.Camera, iters: int, lr: float = 2.5e-3,
                  lam: float = 0.2, opts: gsr.RasterOpts | None = None, exp_avg=None, exp_avg_sq=None,
                  step0: int = 0):
    """`iters` colour-refinement steps on params["colors"] (updated in place).
    frames: list of (pose7 [7], colour [3,H,W], depth [H,W]) device tensors;
    iteration i uses frames[i % len(frames)]. exp_avg / exp_avg_sq: the
    colours' Adam moments (zero tensors when None; updated in place); step0:
    Adam steps already taken with them. Returns (exp_avg, exp_avg_sq, losses
    [iters] device)."""
    colors = params["colors"]
    m = torch.zeros_like(colors) if exp_avg is None else exp_avg
    v = torch.zeros_like(colors) if exp_avg_sq is None else exp_avg_sq
    args = tuple(params[k] for k in gsr.PARAM_GROUPS)
    losses = []
    for i in range(iters):
        pose, tc, td = frames[i % len(frames)]
        c, d, _, st = gsr.render_fwd(*args, pose, camera, opts)
        loss, gC, gD = gsr.loss_map(c, d, tc, td, lam=lam, w_color=1.0, w_depth=0.0)
        g = gsr.render_bwd(st, gC, gD, None, want_params=True, want_pose=False, groups=("colors",))
        st.release()
        gsr.adam_step(colors, m, v, g["colors"], step0 + i + 1, lr)
        losses.append(loss)
    return m, v, torch.cat(losses) if losses else torch.zeros(0, device=colors.device)
