"""Frame-to-model tracking (Sec. 3.4): constant-speed initialisation (Eq. 13)
and pose optimisation (Eq. 14) under the masked tracking loss (Eq. 15),
either as one captured hipGraph per frame or as an eager loop of the same
library calls (the reference the graph is tested against)."""
from __future__ import annotations

import torch

from . import gsr


def overlap_capacity(means, scales, quats, opacities, colors, pose7, camera, opts=None, margin=1.5) -> int:
    """Tile-overlap capacity for a tracking graph: the overlap count at pose7
    times a margin (pose updates within a frame change it little)."""
    _, _, _, st = gsr.render_fwd(means, scales, quats, opacities, colors, pose7, camera, opts)
    K = gsr.state_stats(st)["K"]
    st.release()
    return max(int(K * margin), 4096)


def track_eager(means, scales, quats, opacities, colors, camera, obs_color, obs_depth, pose7, n_iters=100,
                lambda_c=0.5, inlier_mult=50.0, lr_q=5e-4, lr_t=1e-3, betas=(0.9, 0.999), eps=1e-8, opts=None):
    """The tracking loop issued call by call (no graph). Returns (pose7, losses)."""
    pose = pose7.clone()
    state = torch.zeros(20, device=pose.device, dtype=torch.float32)
    losses = []
    for _ in range(n_iters):
        color, depth, alpha, st = gsr.render_fwd(means, scales, quats, opacities, colors, pose, camera, opts)
        loss, gC, gD, _ = gsr.loss_track(color, depth, alpha, obs_color, obs_depth, lambda_c, inlier_mult)
        g = gsr.render_bwd(st, gC, gD, None, want_params=False, want_pose=True)
        st.release()
        gsr.pose_adam_step(pose, state, g["pose7"], lr_q, lr_t, betas[0], betas[1], eps)
        losses.append(loss)
    return pose, torch.cat(losses)


def track_autograd(means, scales, quats, opacities, colors, camera, obs_color, obs_depth, pose7, n_iters=100,
                   lambda_c=0.5, inlier_mult=50.0, lr_q=5e-4, lr_t=1e-3, betas=(0.9, 0.999), eps=1e-8, opts=None):
    """The tracking loop written with torch autograd: the pose is split into a
    quaternion and a translation leaf (one Adam step size each), the render
    and the Eq. 15 loss are the library's (render.render, render.loss_track)
    and loss.backward() runs the library's hand-written adjoint. The Gaussians
    are constants (frozen while tracking, Sec. 3.4). Returns (pose7, losses)."""
    from . import render as R
    q = pose7[:4].detach().clone().requires_grad_(True)
    t = pose7[4:].detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([{"params": [q], "lr": lr_q}, {"params": [t], "lr": lr_t}], betas=betas, eps=eps)
    losses = []
    for _ in range(n_iters):
        opt.zero_grad(set_to_none=True)
        color, depth, alpha = R.render(means, scales, quats, opacities, colors, torch.cat([q, t]), camera, opts)
        loss = R.loss_track(color, depth, alpha, obs_color, obs_depth, lambda_c, inlier_mult)
        loss.backward()
        opt.step()
        losses.append(loss.detach().reshape(1))
    return torch.cat([q, t]).detach(), torch.cat(losses)
