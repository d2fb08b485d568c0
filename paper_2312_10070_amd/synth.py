"""Seeded synthetic inputs for the Gaussian rasterization hot path.

This module only *generates* inputs: Gaussian parameters, camera intrinsics,
poses and ray-cast RGB-D frames of a procedural room. It contains none of the
rasterizer's arithmetic (no projection of Gaussians, no compositing, no
gradients), so both the FP64 oracle and the HIP path can consume it.

The paper evaluates on Replica / TUM-RGBD / ScanNet(++) (Sec. 4, "Datasets");
none of those are available here, so a procedural room stands in for them: an
axis-aligned 6 x 3 x 5 m box room with textured walls and a few boxes on the
floor, seeded the way Sec. 3.2 ("Sub-map Building") and the supplement seed a
sub-map: points back-projected from an RGB-D frame, scales from the nearest
neighbour distance, opacity 0.5, colour from the image.

Conventions: quaternions are (w, x, y, z); a pose7 is (qw, qx, qy, qz, tx, ty,
tz) mapping world to camera; cameras look down +z with +x right and +y down.
All arrays are float32 unless stated.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

IDENTITY_POSE = np.array([1, 0, 0, 0, 0, 0, 0], np.float32)


@dataclass(frozen=True)
class Intrinsics:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    near_z: float = 0.2


C1_CAMERA = Intrinsics(64, 48, 60.0, 60.0, 32.0, 24.0)
MAPPING_CAMERA = Intrinsics(1200, 680, 600.0, 600.0, 600.0, 340.0)
TRACKING_CAMERA = Intrinsics(640, 480, 525.0, 525.0, 320.0, 240.0)


# ----------------------------------------------------------------------------
# small rotation helpers (input generation only)
# ----------------------------------------------------------------------------

def quat_to_matrix(q) -> np.ndarray:
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def matrix_to_quat(R) -> np.ndarray:
    """Unit quaternion (w >= 0) of a rotation matrix (Shepperd's method)."""
    R = np.asarray(R, np.float64)
    tr = np.trace(R)
    if tr > 0:
        s = np.sqrt(tr + 1.0) * 2
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif R[1, 1] > R[2, 2]:
        s = np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    q /= np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def axis_angle_matrix(axis, angle) -> np.ndarray:
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def pose7_from_Rt(R_wc, t_wc) -> np.ndarray:
    return np.concatenate([matrix_to_quat(R_wc), np.asarray(t_wc, np.float64)]).astype(np.float32)


def pose7_to_Rt(p7):
    p7 = np.asarray(p7, np.float64)
    return quat_to_matrix(p7[:4]), p7[4:7].copy()


def camera_pose(center, yaw, pitch) -> np.ndarray:
    """World-to-camera pose7 for a camera at `center` with yaw about -y (up) and pitch."""
    cy_, sy_ = np.cos(yaw), np.sin(yaw)
    cp, sp = np.cos(pitch), np.sin(pitch)
    R_yaw = np.array([[cy_, 0, sy_], [0, 1, 0], [-sy_, 0, cy_]])
    R_pitch = np.array([[1, 0, 0], [0, cp, -sp], [0, sp, cp]])
    R_cw = R_yaw @ R_pitch  # camera axes expressed in world
    R_wc = R_cw.T
    t_wc = -R_wc @ np.asarray(center, np.float64)
    return pose7_from_Rt(R_wc, t_wc)


def perturb_pose(p7, rng, trans_m, rot_deg) -> np.ndarray:
    """Left-compose a rigid motion of exactly `trans_m` metres along a random
    axis and `rot_deg` degrees about another random axis."""
    R, t = pose7_to_Rt(p7)
    a = rng.normal(size=3)
    b = rng.normal(size=3)
    dR = axis_angle_matrix(a, np.deg2rad(rot_deg))
    dt = trans_m * b / np.linalg.norm(b)
    return pose7_from_Rt(dR @ R, dR @ t + dt)


def pose_error(p_est, p_gt):
    """(translation error in metres of the camera centre, rotation error in degrees)."""
    Re, te = pose7_to_Rt(p_est)
    Rg, tg = pose7_to_Rt(p_gt)
    ce = -Re.T @ te
    cg = -Rg.T @ tg
    dR = Re @ Rg.T
    ang = np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1.0, 1.0)))
    return float(np.linalg.norm(ce - cg)), float(ang)


def random_unit_quats(rng, n) -> np.ndarray:
    q = rng.normal(size=(n, 4))
    return (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)


# ----------------------------------------------------------------------------
# config C1: 1,000 random Gaussians in front of a 64 x 48 camera
# ----------------------------------------------------------------------------

def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def c1_raw(seed: int, n: int = 1000) -> dict:
    """Raw (unactivated) parameters: means, log-scales, quats, logit-opacity, colours."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(1, 5, n)], 1)
    log_scales = rng.normal(-3.0, 0.3, size=(n, 3))
    quats = rng.normal(size=(n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    logit_o = rng.normal(0.0, 1.0, size=n)
    colors = rng.uniform(0, 1, size=(n, 3))
    return dict(means=means, log_scales=log_scales, quats=quats, logit_opacities=logit_o, colors=colors)


def activate(raw: dict) -> dict:
    """Activated float32 parameters as the renderer takes them."""
    q = raw["quats"] / np.linalg.norm(raw["quats"], axis=1, keepdims=True)
    return dict(
        means=np.ascontiguousarray(raw["means"], np.float32),
        scales=np.ascontiguousarray(np.exp(raw["log_scales"]), np.float32),
        quats=np.ascontiguousarray(q, np.float32),
        opacities=np.ascontiguousarray(_sigmoid(raw["logit_opacities"]), np.float32),
        colors=np.ascontiguousarray(raw["colors"], np.float32),
    )


def perturb_raw(raw: dict, seed: int, std: float = 0.01) -> dict:
    rng = np.random.default_rng(seed + 7919)
    return {k: v + rng.normal(0.0, std, size=v.shape) for k, v in raw.items()}


def c1_inputs(seed: int = 0, n: int = 1000) -> dict:
    """C1: Gaussians, the perturbed target Gaussians, identity pose, camera."""
    raw = c1_raw(seed, n)
    return dict(gaussians=activate(raw), target_gaussians=activate(perturb_raw(raw, seed)),
                pose7=IDENTITY_POSE.copy(), camera=C1_CAMERA)


# ----------------------------------------------------------------------------
# procedural room
# ----------------------------------------------------------------------------

ROOM_MIN = np.array([-3.0, -1.5, -2.5])
ROOM_MAX = np.array([3.0, 1.5, 2.5])


@dataclass
class Room:
    boxes_min: np.ndarray  # [B,3]
    boxes_max: np.ndarray  # [B,3]
    base_colors: np.ndarray  # [6 + B, 3] per surface
    phase: np.ndarray  # [6 + B, 2]


def make_room(seed: int, n_boxes: int = 4, scale_jitter: float = 0.0) -> Room:
    rng = np.random.default_rng(seed + 104729)
    bmin, bmax = [], []
    for _ in range(n_boxes):
        size = rng.uniform(0.3, 1.0, 3)
        cx = rng.uniform(ROOM_MIN[0] + 0.6, ROOM_MAX[0] - 0.6 - size[0])
        cz = rng.uniform(ROOM_MIN[2] + 0.6, ROOM_MAX[2] - 0.6 - size[2])
        lo = np.array([cx, ROOM_MAX[1] - size[1], cz])  # resting on the floor (y = +1.5 is down)
        bmin.append(lo)
        bmax.append(lo + size)
    nsurf = 6 + n_boxes
    return Room(np.array(bmin).reshape(-1, 3), np.array(bmax).reshape(-1, 3),
                rng.uniform(0.15, 0.85, (nsurf, 3)), rng.uniform(0, 2 * np.pi, (nsurf, 2)))


def _texture(room: Room, pts: np.ndarray, surf: np.ndarray, normal_axis: np.ndarray) -> np.ndarray:
    """Procedural colour: base colour + 0.1 m checker + two sinusoids, in [0,1]."""
    # in-plane coordinates: the two axes other than the surface normal
    ax = np.stack([(normal_axis + 1) % 3, (normal_axis + 2) % 3], 1)
    u = np.take_along_axis(pts, ax[:, :1], 1)[:, 0]
    v = np.take_along_axis(pts, ax[:, 1:], 1)[:, 0]
    checker = ((np.floor(u / 0.1) + np.floor(v / 0.1)) % 2) * 2 - 1
    ph = room.phase[surf]
    s1 = np.sin(2 * np.pi * u / 0.37 + ph[:, 0])
    s2 = np.sin(2 * np.pi * v / 0.23 + ph[:, 1])
    base = room.base_colors[surf]
    col = base + 0.08 * checker[:, None] + 0.06 * s1[:, None] * np.array([1.0, 0.6, 0.2]) \
        + 0.06 * s2[:, None] * np.array([0.2, 0.5, 1.0])
    return np.clip(col, 0.0, 1.0)


def raycast(room: Room, cam: Intrinsics, pose7, pixels_xy=None):
    """Ray-cast the room. Returns (depth [M], color [M,3], world points [M,3]) for the
    given continuous pixel coordinates [M,2] (default: every pixel centre)."""
    R_wc, t_wc = pose7_to_Rt(pose7)
    R_cw = R_wc.T
    c = -R_cw @ t_wc
    if pixels_xy is None:
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        pixels_xy = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.float64)
    d_cam = np.stack([(pixels_xy[:, 0] - cam.cx) / cam.fx, (pixels_xy[:, 1] - cam.cy) / cam.fy,
                      np.ones(len(pixels_xy))], 1)
    d = d_cam @ R_cw.T  # world direction; ray parameter == camera depth
    M = len(d)
    best = np.full(M, np.inf)
    surf = np.zeros(M, np.int64)
    naxis = np.zeros(M, np.int64)
    with np.errstate(divide="ignore", invalid="ignore"):
        # room walls: the ray exits through the nearest plane with t > 0
        for axis in range(3):
            for side, bound in ((0, ROOM_MIN[axis]), (1, ROOM_MAX[axis])):
                t = (bound - c[axis]) / d[:, axis]
                ok = (t > 1e-6) & (t < best)
                best = np.where(ok, t, best)
                surf = np.where(ok, 2 * axis + side, surf)
                naxis = np.where(ok, axis, naxis)
        # boxes (slab test)
        for b in range(len(room.boxes_min)):
            t0 = (room.boxes_min[b] - c) / d
            t1 = (room.boxes_max[b] - c) / d
            tmin = np.minimum(t0, t1)
            tmax = np.maximum(t0, t1)
            tn = np.max(tmin, axis=1)
            tf = np.min(tmax, axis=1)
            hit = (tn <= tf) & (tn > 1e-6) & (tn < best)
            ax = np.argmax(tmin, axis=1)
            best = np.where(hit, tn, best)
            surf = np.where(hit, 6 + b, surf)
            naxis = np.where(hit, ax, naxis)
    pts = c + best[:, None] * d
    col = _texture(room, pts, surf, naxis)
    return best, col, pts


def render_frame(room: Room, cam: Intrinsics, pose7):
    """Ground-truth RGB-D frame: color [3,H,W] and depth [H,W] (float32)."""
    depth, col, _ = raycast(room, cam, pose7)
    H, W = cam.height, cam.width
    return (np.ascontiguousarray(col.T.reshape(3, H, W), np.float32),
            np.ascontiguousarray(depth.reshape(H, W), np.float32))


def random_view(rng) -> np.ndarray:
    lo = ROOM_MIN + 0.2 * (ROOM_MAX - ROOM_MIN)
    hi = ROOM_MAX - 0.2 * (ROOM_MAX - ROOM_MIN)
    center = rng.uniform(lo, hi)
    return camera_pose(center, rng.uniform(-np.pi, np.pi), np.deg2rad(rng.uniform(-15, 15)))


def open_view(room: Room, rng, cam: Intrinsics, tries: int = 12) -> np.ndarray:
    """A random view that looks across the room: of `tries` random views, the one
    with the largest median depth on a coarse ray-cast (an indoor scan views
    the room, not a wall at arm's length)."""
    small = Intrinsics(cam.width // 16, cam.height // 16, cam.fx / 16, cam.fy / 16, cam.cx / 16, cam.cy / 16)
    best, best_d = None, -1.0
    for _ in range(tries):
        v = random_view(rng)
        d, _, _ = raycast(room, small, v)
        med = float(np.median(d))
        if med > best_d:
            best, best_d = v, med
    return best


def _nn_distance(pts: np.ndarray) -> np.ndarray:
    from scipy.spatial import cKDTree
    tree = cKDTree(pts)
    d, _ = tree.query(pts, k=2)
    return np.maximum(d[:, 1], 1e-4)


def seed_gaussians(room: Room, cam: Intrinsics, views, n: int, rng, depth_noise: float = 0.005) -> dict:
    """Back-project `n` uniformly sampled pixels of the given views (noisy depth) into
    Gaussians: NN-distance anisotropic scales, random rotations, opacity 0.5,
    colour from the noise-free hit."""
    per = [n // len(views) + (1 if i < n % len(views) else 0) for i in range(len(views))]
    means, cols = [], []
    for pose, m in zip(views, per):
        idx = rng.choice(cam.width * cam.height, size=m, replace=m > cam.width * cam.height)
        xy = np.stack([idx % cam.width, idx // cam.width], 1).astype(np.float64)
        xy += rng.uniform(-0.5, 0.5, xy.shape)
        depth, col, _ = raycast(room, cam, pose, xy)
        depth = depth + rng.normal(0.0, depth_noise, depth.shape)
        R_wc, t_wc = pose7_to_Rt(pose)
        pc = np.stack([(xy[:, 0] - cam.cx) / cam.fx * depth, (xy[:, 1] - cam.cy) / cam.fy * depth, depth], 1)
        pw = (pc - t_wc) @ R_wc  # R_wc^T (pc - t)
        means.append(pw)
        cols.append(col)
    means = np.concatenate(means)
    cols = np.concatenate(cols)
    dnn = _nn_distance(means)
    scales = dnn[:, None] * np.exp(rng.normal(0.0, 0.3, size=(len(means), 3)))
    return dict(
        means=np.ascontiguousarray(means, np.float32),
        scales=np.ascontiguousarray(scales, np.float32),
        quats=random_unit_quats(rng, len(means)),
        opacities=np.full(len(means), 0.5, np.float32),
        colors=np.ascontiguousarray(cols, np.float32),
    )


def mapping_inputs(seed: int = 0, n: int = 200_000, cam: Intrinsics = MAPPING_CAMERA) -> dict:
    """C2 / headline: one view of the room, `n` Gaussians seeded from it, RGB-D target."""
    rng = np.random.default_rng(seed)
    room = make_room(seed)
    pose = open_view(room, rng, cam)
    g = seed_gaussians(room, cam, [pose], n, rng)
    color, depth = render_frame(room, cam, pose)
    return dict(gaussians=g, pose7=pose, camera=cam, target_color=color, target_depth=depth)


def image_pair(seed: int = 0, cam: Intrinsics = MAPPING_CAMERA, noise: float = 0.02):
    """Two colour images [3,H,W] of the room for the mapping colour loss: the
    ground-truth frame at a view, and a stand-in for a render (the frame at that
    view moved by 2 cm / 1 degree, plus N(0, noise) clipped to [0, 1])."""
    rng = np.random.default_rng(seed)
    room = make_room(seed)
    pose = open_view(room, rng, MAPPING_CAMERA)  # the view is chosen at a fixed probe size
    tgt, _ = render_frame(room, cam, pose)
    near, _ = render_frame(room, cam, perturb_pose(pose, rng, 0.02, 1.0))
    ren = np.clip(near + rng.normal(0.0, noise, near.shape), 0.0, 1.0).astype(np.float32)
    return ren, tgt


def tracking_inputs(seed: int = 0, n: int = 500_000, cam: Intrinsics = TRACKING_CAMERA, n_views: int = 5,
                    trans_m: float = 0.02, rot_deg: float = 1.0) -> dict:
    """C3: sub-map seeded from views near the ground-truth pose, GT pose, perturbed init."""
    rng = np.random.default_rng(seed)
    room = make_room(seed)
    gt = open_view(room, rng, cam)
    views = [gt] + [perturb_pose(gt, rng, rng.uniform(0, 0.3), rng.uniform(0, 10)) for _ in range(n_views - 1)]
    g = seed_gaussians(room, cam, views, n, rng)
    init = perturb_pose(gt, rng, trans_m, rot_deg)
    return dict(gaussians=g, gt_pose7=gt, init_pose7=init, camera=cam, room=room)


def batched_inputs(seed: int = 0, n: int = 1_000_000, cam: Intrinsics = MAPPING_CAMERA, n_views: int = 8,
                   n_seed_views: int = 16, n_candidates: int = 48) -> dict:
    """C4: a sub-map seeded from 16 views around one spot of the room (within
    0.4 m, turned up to 25 degrees either way from a base heading) and
    candidate keyframes from that spot turned by 0 to 180 degrees from the
    base heading (and moved up to 0.3 m): their visible fractions of the
    sub-map spread from most of it to little of it. The caller picks the 8
    keyframes from `candidate_views`."""
    rng = np.random.default_rng(seed)
    room = make_room(seed)
    lo = ROOM_MIN + 0.3 * (ROOM_MAX - ROOM_MIN)
    hi = ROOM_MAX - 0.3 * (ROOM_MAX - ROOM_MIN)
    center = rng.uniform(lo, hi)
    yaw0 = rng.uniform(-np.pi, np.pi)

    def view(max_move, yaw_off, pitch_deg):
        d = rng.normal(size=3)
        c = center + max_move * rng.uniform() * d / np.linalg.norm(d)
        return camera_pose(c, yaw0 + yaw_off, np.deg2rad(pitch_deg))

    seed_views = [view(0.4, np.deg2rad(rng.uniform(-25, 25)), rng.uniform(-10, 10)) for _ in range(n_seed_views)]
    g = seed_gaussians(room, cam, seed_views, n, rng)
    offsets = np.deg2rad(np.linspace(0, 180, n_candidates)) * rng.choice([-1, 1], n_candidates)
    candidates = [view(0.3, off, rng.uniform(-10, 10)) for off in offsets]
    return dict(gaussians=g, candidate_views=candidates, camera=cam, room=room, n_views=n_views)
