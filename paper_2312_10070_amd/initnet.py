"""Learned tracking-pose initialisation.

A small CNN (four 3x3 stride-2 convolutions, 64 channels, ReLU, global average
pooling, linear head; BF16 matrix-core kernels in libgsr) maps the render at
the current pose estimate and the observed RGB-D frame (both downsampled to
160 x 120) to the twist (rho, phi) that takes the estimate to the camera pose.
The paper initialises tracking with a constant-speed model (Eq. 13) and,
in its supplement, lets an alternative initialiser take over when the loss
says it is better; here the network's proposal replaces the constant-speed
pose only when the tracking loss (Eq. 15) at the proposal is lower.

Training pairs are rendered by the project's own forward kernels from random
procedural rooms: the observation is the render at the true pose, the input
render is at a pose perturbed by up to 5 cm / 3 degrees, and the label is the
twist back to the true pose.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gsr, synth

CHANNELS = 64
IN_CHANNELS = (8, 64, 64, 64)
DEPTH_SCALE = 0.25
# the label scale (metres for rho, radians for phi) the loss divides by
LABEL_SCALE = (0.02, 0.02, 0.02, 0.02, 0.02, 0.02)


def kp(c: int) -> int:
    return ((9 * c + 31) // 32) * 32


def layout():
    """[(name, shape, offset)] of the flat FP32 parameter vector."""
    out, off = [], 0
    for l, c in enumerate(IN_CHANNELS):
        out.append((f"w{l}", (CHANNELS, kp(c)), off)); off += CHANNELS * kp(c)
        out.append((f"b{l}", (CHANNELS,), off)); off += CHANNELS
    out.append(("wfc", (6, CHANNELS), off)); off += 6 * CHANNELS
    out.append(("bfc", (6,), off)); off += 6
    return out, off


def init_params(seed: int) -> np.ndarray:
    """He-normal convolution weights (zero pad columns), small head."""
    rng = np.random.default_rng(seed)
    lay, n = layout()
    flat = np.zeros(n, np.float32)
    for name, shape, off in lay:
        size = int(np.prod(shape))
        if name.startswith("w") and name != "wfc":
            l = int(name[1:])
            c = IN_CHANNELS[l]
            w = np.zeros(shape, np.float32)
            w[:, :9 * c] = rng.normal(0, np.sqrt(2.0 / (9 * c)), size=(shape[0], 9 * c))
            flat[off:off + size] = w.ravel()
        elif name == "wfc":
            flat[off:off + size] = rng.normal(0, 0.01, size=size)
    return flat


def to_oihw(flat: np.ndarray) -> dict:
    """Flat packed vector -> {w_l [64, C, 3, 3], b_l, wfc, bfc} (float64)."""
    lay, _ = layout()
    out = {}
    for name, shape, off in lay:
        v = np.asarray(flat[off:off + int(np.prod(shape))], np.float64).reshape(shape)
        if name.startswith("w") and name != "wfc":
            c = IN_CHANNELS[int(name[1:])]
            v = v[:, :9 * c].reshape(CHANNELS, 3, 3, c).transpose(0, 3, 1, 2)
        out[name] = v
    return out


def pack_grads_oihw(g: dict) -> np.ndarray:
    """Inverse of to_oihw (for comparing gradients in the packed layout)."""
    lay, n = layout()
    flat = np.zeros(n)
    for name, shape, off in lay:
        v = np.asarray(g[name], np.float64)
        if name.startswith("w") and name != "wfc":
            c = IN_CHANNELS[int(name[1:])]
            p = np.zeros(shape)
            p[:, :9 * c] = v.transpose(0, 2, 3, 1).reshape(CHANNELS, 9 * c)
            v = p
        flat[off:off + int(np.prod(shape))] = v.ravel()
    return flat


def random_twist(rng, max_t=0.05, max_deg=3.0) -> np.ndarray:
    """A twist with a translation uniform in a ball of radius max_t and a
    rotation uniform in angle up to max_deg about a uniform axis."""
    d = rng.normal(size=3); d /= np.linalg.norm(d)
    rho = d * max_t * rng.uniform() ** (1 / 3)
    a = rng.normal(size=3); a /= np.linalg.norm(a)
    phi = a * np.deg2rad(max_deg) * rng.uniform()
    return np.concatenate([rho, phi])


def inverse_twist(xi: np.ndarray) -> np.ndarray:
    """The twist whose left perturbation undoes exp(xi^)."""
    from scipy.spatial.transform import Rotation
    E = Rotation.from_rotvec(xi[3:]).as_matrix()
    return np.concatenate([-(E.T @ xi[:3]), -xi[3:]])


def generate_pairs(n_pairs: int, seed: int, cam: synth.Intrinsics, gaussians_per_room=20_000, pairs_per_view=32,
                   views_per_room=4, max_t=0.05, max_deg=3.0):
    """Render n_pairs (input, label) samples. Returns (x BF16 [N,120,160,8],
    labels FP32 [N,6]) on the device."""
    rng = np.random.default_rng(seed)
    camera = gsr.camera_from(cam)
    x = torch.empty((n_pairs, 120, 160, 8), device="cuda", dtype=torch.bfloat16)
    labels = np.zeros((n_pairs, 6), np.float32)
    i = 0
    room_id = 0
    while i < n_pairs:
        room = synth.make_room(seed * 100003 + room_id)
        room_id += 1
        views = [synth.random_view(rng) for _ in range(views_per_room)]
        g = synth.seed_gaussians(room, cam, views, gaussians_per_room, rng)
        gd = {k: torch.from_numpy(v).cuda() for k, v in g.items()}
        args = (gd["means"], gd["scales"], gd["quats"], gd["opacities"], gd["colors"])
        for gt in views:
            gt_d = torch.from_numpy(gt).cuda()
            oc, od, _, st = gsr.render_fwd(*args, gt_d, camera)
            st.release()
            for _ in range(pairs_per_view):
                if i >= n_pairs:
                    break
                xi = random_twist(rng, max_t, max_deg)  # label: from the perturbed pose back to gt
                pert = gsr.pose_apply_twist(gt_d, torch.from_numpy(inverse_twist(xi).astype(np.float32)).cuda())
                rc, rd, _, st = gsr.render_fwd(*args, pert, camera)
                st.release()
                gsr.pack_rgbd_pair(rc, rd, oc, od, x[i], DEPTH_SCALE)
                labels[i] = xi
                i += 1
    return x, torch.from_numpy(labels).cuda()


def train(net: gsr.InitNet, x, labels, steps: int, batch: int, lr: float = 1e-3, seed: int = 0, log_every: int = 0):
    """Adam on the MSE of the scaled twist; returns the per-step losses."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    scale = torch.tensor(LABEL_SCALE, device="cuda", dtype=torch.float32)
    losses = []
    N = x.shape[0]
    for s in range(steps):
        idx = torch.randint(0, N, (batch,), generator=g).cuda()
        net.set_input(x.index_select(0, idx).contiguous())
        net.forward(batch)
        loss = net.backward(batch, labels.index_select(0, idx).contiguous(), scale)
        net.adam(lr * (0.5 * (1 + np.cos(np.pi * s / steps))) + 1e-5)
        losses.append(loss)
        if log_every and s % log_every == 0:
            print(f"step {s} loss {loss.item():.4f}", flush=True)
    return torch.cat(losses).cpu().numpy()


def predict(net: gsr.InitNet, x) -> torch.Tensor:
    """Twists for packed inputs x [B,120,160,8] (B <= max_batch)."""
    net.set_input(x.contiguous())
    return net.forward(x.shape[0])


def propose(net: gsr.InitNet, gaussians: tuple, camera: gsr.Camera, obs_color, obs_depth, pose7,
            lambda_c=0.5, inlier_mult=50.0, opts=None):
    """Learned initialisation with a loss-judged fallback: render at pose7,
    predict a twist, and keep the proposal only if the tracking loss (Eq. 15)
    there is lower than at pose7. Returns (pose, used_proposal, loss_pose7, loss_proposal)."""
    rc, rd, ra, st = gsr.render_fwd(*gaussians, pose7, camera, opts)
    st.release()
    l0 = gsr.loss_track(rc, rd, ra, obs_color, obs_depth, lambda_c, inlier_mult)[0]
    buf = torch.empty((1, 120, 160, 8), device="cuda", dtype=torch.bfloat16)
    gsr.pack_rgbd_pair(rc, rd, obs_color, obs_depth, buf[0], DEPTH_SCALE)
    xi = predict(net, buf)[0].contiguous()
    prop = gsr.pose_apply_twist(pose7, xi)
    pc, pd, pa, st = gsr.render_fwd(*gaussians, prop, camera, opts)
    st.release()
    l1 = gsr.loss_track(pc, pd, pa, obs_color, obs_depth, lambda_c, inlier_mult)[0]
    use = bool(l1.item() < l0.item())
    return (prop if use else pose7), use, float(l0.item()), float(l1.item())
