"""Learned tracking-pose initialisation.

A small CNN (four 3x3 stride-2 convolutions, 64 channels, ReLU, moment
pooling, linear head; BF16 matrix-core kernels in libgsr) maps the render at
the current pose estimate and the observed RGB-D frame (packed as the render
and the observed-minus-rendered residual, downsampled to 160 x 120) to the
twist (rho, phi) that takes the estimate to the camera pose. Moment pooling
keeps, per channel, the mean of the last feature map and its means weighted
by the horizontal and vertical position: a forward motion or a roll moves
image content radially or around the centre, which a plain average cancels.
The paper initialises tracking with a constant-speed model (Eq. 13) and,
in its supplement, lets an alternative initialiser take over when the loss
says it is better; here the network's proposal replaces the constant-speed
pose only when the tracking loss (Eq. 15) at the proposal is lower.

Training pairs are rendered by the project's own forward kernels from random
procedural scenes built like tracking sub-maps: the observation is the render
at the true pose, the input render is at a pose perturbed by up to 5 cm / 3
degrees, and the label is the twist back to the true pose.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gsr, synth

CHANNELS = 64
IN_CHANNELS = (8, 64, 64, 64)
HEAD_IN = 3 * CHANNELS  # moment pooling: mean, x-weighted and y-weighted means per channel
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
    out.append(("wfc", (6, HEAD_IN), off)); off += 6 * HEAD_IN
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


def scene_for_pairs(args):
    """One training scene (CPU only, run in worker processes): a random room
    (boxes, textures), a base view looking across it, a
    sub-map seeded from the base view and four views within 0.3 m / 10
    degrees of it (as a tracking sub-map is), and the observation views, also
    within 0.3 m / 10 degrees of the base."""
    seed, cam, n_gaussians, n_obs = args
    rng = np.random.default_rng(seed)
    room = synth.make_room(seed)
    base = synth.open_view(room, rng, cam)
    seeds = [base] + [synth.perturb_pose(base, rng, rng.uniform(0, 0.3), rng.uniform(0, 10)) for _ in range(4)]
    g = synth.seed_gaussians(room, cam, seeds, n_gaussians, rng)
    obs = [synth.perturb_pose(base, rng, rng.uniform(0, 0.3), rng.uniform(0, 10)) for _ in range(n_obs)]
    return g, obs


def generate_pairs(n_pairs: int, seed: int, cam: synth.Intrinsics, gaussians_per_scene=150_000,
                   obs_views_per_scene=16, pairs_per_view=32, max_t=0.05, max_deg=3.0, workers=8, log=None):
    """Render n_pairs (input, label) samples from procedural scenes built like
    tracking sub-maps (scene_for_pairs, seeded on `workers` CPU processes).
    Per observation view: the observed frame is the render at that view, the
    input render is at the view perturbed by up to max_t / max_deg, and the
    label is the twist from the perturbed pose back to the view. Returns
    (x BF16 [N,120,160,8], labels FP32 [N,6]) on the device."""
    import multiprocessing as mp
    rng = np.random.default_rng(seed)
    camera = gsr.camera_from(cam)
    per_scene = obs_views_per_scene * pairs_per_view
    n_scenes = (n_pairs + per_scene - 1) // per_scene
    jobs = [(seed * 100003 + k, cam, gaussians_per_scene, obs_views_per_scene) for k in range(n_scenes)]
    x = torch.empty((n_pairs, 120, 160, 8), device="cuda", dtype=torch.bfloat16)
    labels = np.zeros((n_pairs, 6), np.float32)
    i = 0
    with mp.get_context("spawn").Pool(max(1, workers)) as pool:
        for g, obs in pool.imap(scene_for_pairs, jobs):
            gd = {k: torch.from_numpy(v).cuda() for k, v in g.items()}
            args = (gd["means"], gd["scales"], gd["quats"], gd["opacities"], gd["colors"])
            for view in obs:
                if i >= n_pairs:
                    break
                v_d = torch.from_numpy(view.astype(np.float32)).cuda()
                oc, od, _, st = gsr.render_fwd(*args, v_d, camera)
                st.release()
                for _ in range(pairs_per_view):
                    if i >= n_pairs:
                        break
                    xi = random_twist(rng, max_t, max_deg)  # label: from the perturbed pose back to the view
                    pert = gsr.pose_apply_twist(v_d, torch.from_numpy(inverse_twist(xi).astype(np.float32)).cuda())
                    rc, rd, _, st = gsr.render_fwd(*args, pert, camera)
                    st.release()
                    gsr.pack_rgbd_pair(rc, rd, oc, od, x[i], DEPTH_SCALE)
                    labels[i] = xi
                    i += 1
            if log:
                log(i)
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
            lambda_c=0.5, inlier_mult=50.0, opts=None, max_steps: int = 1):
    """Learned initialisation with a loss-judged fallback: render at the
    current pose, predict a twist, and move to the proposal only if the
    tracking loss (Eq. 15) there is lower; repeated up to max_steps times (each
    step starts from the pose the last one kept) and stopped at the first
    proposal the loss rejects. Returns (pose, proposals kept, loss at pose7,
    loss at the returned pose)."""
    buf = torch.empty((1, 120, 160, 8), device="cuda", dtype=torch.bfloat16)
    rc, rd, ra, st = gsr.render_fwd(*gaussians, pose7, camera, opts)
    st.release()
    l_cur = float(gsr.loss_track(rc, rd, ra, obs_color, obs_depth, lambda_c, inlier_mult)[0].item())
    l0 = l_cur
    pose, kept = pose7, 0
    for _ in range(max_steps):
        gsr.pack_rgbd_pair(rc, rd, obs_color, obs_depth, buf[0], DEPTH_SCALE)
        xi = predict(net, buf)[0].contiguous()
        prop = gsr.pose_apply_twist(pose, xi)
        pc, pd, pa, st = gsr.render_fwd(*gaussians, prop, camera, opts)
        st.release()
        l_prop = float(gsr.loss_track(pc, pd, pa, obs_color, obs_depth, lambda_c, inlier_mult)[0].item())
        if not l_prop < l_cur:
            break
        pose, l_cur, kept = prop, l_prop, kept + 1
        rc, rd = pc, pd
    return pose, kept, l0, l_cur
