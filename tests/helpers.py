"""Shared test helpers: an independent numpy route to the paper's quantities
(used only to pin the oracle), finite differences, and tolerance checks.

Nothing here imports the HIP library; GPU tests import it themselves.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

import oracle
from paper_2312_10070_amd import synth


def cam_of(intr: synth.Intrinsics, bg=(0.0, 0.0, 0.0)) -> oracle.Camera:
    return oracle.Camera(intr.width, intr.height, intr.fx, intr.fy, intr.cx, intr.cy, intr.near_z, tuple(bg))


def scipy_R(q_wxyz) -> np.ndarray:
    q = np.asarray(q_wxyz, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def gl_projection(cam: oracle.Camera, near=0.01, far=100.0) -> np.ndarray:
    """OpenGL-style 4x4 projection (the P of Eq. 1) for an OpenCV-style camera,
    acting on GL eye coordinates (x, -y, -z)."""
    W, H = cam.width, cam.height
    return np.array([
        [2 * cam.fx / W, 0, 1 - 2 * cam.cx / W, 0],
        [0, 2 * cam.fy / H, 2 * cam.cy / H - 1, 0],
        [0, 0, -(far + near) / (far - near), -2 * far * near / (far - near)],
        [0, 0, -1, 0],
    ])


def project_gl(mu_world, pose7, cam: oracle.Camera) -> np.ndarray:
    """Eq. 1 written the paper's way: pi(P (T_wc mu_h)), returning pixel (u, v)."""
    T = np.eye(4)
    T[:3, :3] = scipy_R(np.asarray(pose7[:4]) / np.linalg.norm(pose7[:4]))
    T[:3, 3] = pose7[4:7]
    xc = T @ np.append(np.asarray(mu_world, np.float64), 1.0)
    eye_gl = np.array([xc[0], -xc[1], -xc[2], 1.0])
    clip = gl_projection(cam) @ eye_gl
    ndc = clip[:3] / clip[3]
    return np.array([(ndc[0] + 1) * cam.width / 2, (1 - ndc[1]) * cam.height / 2])


def numeric_jacobian(f, x, h=1e-6):
    x = np.asarray(x, np.float64)
    f0 = np.asarray(f(x))
    J = np.zeros((f0.size, x.size))
    for i in range(x.size):
        e = np.zeros_like(x)
        e[i] = h
        J[:, i] = (np.asarray(f(x + e)) - np.asarray(f(x - e))).ravel() / (2 * h)
    return J


def ewa_cov_reference(mu, scale, q, pose7, cam: oracle.Camera, lowpass) -> np.ndarray:
    """Sigma' of Eq. 2 by an independent route: scipy rotations and a numeric
    Jacobian of the pixel projection at the camera-space mean (no clamping)."""
    Rg = scipy_R(np.asarray(q) / np.linalg.norm(q))
    Sigma = Rg @ np.diag(np.asarray(scale, np.float64) ** 2) @ Rg.T
    Rp = scipy_R(np.asarray(pose7[:4]) / np.linalg.norm(pose7[:4]))
    x = Rp @ np.asarray(mu, np.float64) + np.asarray(pose7[4:7], np.float64)
    pix = lambda p: np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])
    J = numeric_jacobian(pix, x, 1e-7)
    return J @ (Rp @ Sigma @ Rp.T) @ J.T + lowpass * np.eye(2)


def brute_force_render(g: dict, pose7, cam: oracle.Camera, opts: oracle.Opts):
    """Independent per-pixel compositing (Eq. 3, 4, 6) over all Gaussians in
    depth order, built on scipy rotations, the GL projection of Eq. 1, a numeric
    Jacobian for Eq. 2 and numpy's matrix inverse. Small inputs only."""
    n = len(g["means"])
    recs = []
    Rp = scipy_R(np.asarray(pose7[:4]) / np.linalg.norm(pose7[:4]))
    for k in range(n):
        mu = np.asarray(g["means"][k], np.float64)
        x = Rp @ mu + np.asarray(pose7[4:7], np.float64)
        if x[2] <= cam.near_z:
            continue
        uv = project_gl(mu, pose7, cam)
        S = ewa_cov_reference(mu, g["scales"][k], g["quats"][k], pose7, cam, opts.lowpass)
        recs.append((x[2], k, uv, np.linalg.inv(S), float(g["opacities"][k]), np.asarray(g["colors"][k], np.float64)))
    recs.sort(key=lambda r: (r[0], r[1]))
    H, W = cam.height, cam.width
    C = np.zeros((3, H, W)); D = np.zeros((H, W)); A = np.zeros((H, W))
    for py in range(H):
        for px in range(W):
            T = 1.0
            c = np.zeros(3); d = 0.0
            for z, k, uv, Ainv, o, col in recs:
                delta = np.array([px, py], np.float64) - uv
                sigma = 0.5 * delta @ Ainv @ delta
                a = min(opts.alpha_max, o * np.exp(-sigma))
                if a < opts.alpha_min:
                    continue
                Tn = T * (1 - a)
                if Tn < opts.T_min:
                    break
                c += col * a * T
                d += z * a * T
                T = Tn
            C[:, py, px] = c + T * np.asarray(cam.bg)
            D[py, px] = d
            A[py, px] = 1 - T
    return C, D, A


def left_perturb_pose(pose7, xi):
    """exp(xi^) T for xi = (rho, phi): R' = Exp(phi) R, t' = Exp(phi) t + rho.
    The rotation of the perturbation uses scipy's rotation vector."""
    R = scipy_R(np.asarray(pose7[:4]) / np.linalg.norm(pose7[:4]))
    t = np.asarray(pose7[4:7], np.float64)
    dR = Rotation.from_rotvec(np.asarray(xi[3:6], np.float64)).as_matrix()
    Rn = dR @ R
    tn = dR @ t + np.asarray(xi[:3], np.float64)
    qx, qy, qz, qw = Rotation.from_matrix(Rn).as_quat()
    q = np.array([qw, qx, qy, qz])
    if np.dot(q, np.asarray(pose7[:4])) < 0:
        q = -q
    return np.concatenate([q * np.linalg.norm(pose7[:4]), tn])


# Admission categories of the gradient bar, in the order the tolerance terms are
# added: plain relative error, then the floor of summed term magnitudes
# (without, then with the transmittance condition number kappa), then the
# slack of ambiguous decisions and screen-position rounding, then the block
# floor. Each element is counted in the first category whose cumulative
# tolerance admits it.
AUDIT_KEYS = ("rel", "floor_plain", "floor_kappa", "slack", "block", "fail")
AUDIT_LOG: list = []


def grad_audit(got, ref, aref, aref_plain=None, slack=None, rel=1e-3, floor=1e-5, block_floor=1e-6) -> dict:
    """Per-category element counts of the gradient bar (see AUDIT_KEYS)."""
    got = np.asarray(got, np.float64); ref = np.asarray(ref, np.float64)
    err = np.abs(got - ref)
    aref = np.asarray(aref, np.float64)
    aplain = aref if aref_plain is None else np.asarray(aref_plain, np.float64)
    t = [rel * np.abs(ref)]
    t.append(t[0] + floor * aplain)
    t.append(t[0] + floor * aref)
    t.append(t[2] + (0.0 if slack is None else np.asarray(slack, np.float64)))
    t.append(t[3] + (block_floor * np.abs(ref).max() if ref.size else 0.0))
    cat = np.full(err.shape, len(t), np.int64)
    for i in range(len(t) - 1, -1, -1):
        cat = np.where(err <= t[i], i, cat)
    counts = {k: int((cat == i).sum()) for i, k in enumerate(AUDIT_KEYS)}
    counts["n"] = int(err.size)
    # elements where either side is non-zero (an element both sides leave at
    # exactly zero passes the relative bar trivially)
    counts["nz"] = int(((ref != 0) | (got != 0)).sum())
    return counts


def check_grad(name, got, ref, aref, slack=None, rel=1e-3, floor=1e-5, block_floor=1e-6, max_bad=0,
               aref_plain=None, case=None):
    """|got - ref| <= rel |ref| + floor * aref + block_floor * max|ref| + slack,
    elementwise. The block floor covers FP32 rounding in chains that cancel
    exactly in FP64 (e.g. the quaternion gradient of an isotropic Gaussian).
    Returns the audit of the bar (grad_audit) and records it in AUDIT_LOG."""
    got = np.asarray(got, np.float64); ref = np.asarray(ref, np.float64)
    tol = rel * np.abs(ref) + floor * np.asarray(aref, np.float64)
    if ref.size:
        tol = tol + block_floor * np.abs(ref).max()
    if slack is not None:
        tol = tol + np.asarray(slack, np.float64)
    err = np.abs(got - ref)
    bad = err > tol
    nbad = int(bad.sum())
    audit = grad_audit(got, ref, aref, aref_plain, slack, rel, floor, block_floor)
    AUDIT_LOG.append(dict(case=case, group=name, **audit))
    if nbad > max_bad:
        i = np.unravel_index(np.argmax(np.where(bad, err / np.maximum(tol, 1e-300), 0)), err.shape)
        raise AssertionError(f"{name}: {nbad} elements out of tolerance; worst at {i}: got {got[i]!r} "
                             f"ref {ref[i]!r} tol {tol[i]!r}")
    return audit


def check_grad_ref(name, got, ref: dict, case=None, **kw):
    """check_grad of one parameter group against an oracle.backward result."""
    return check_grad(name, got, ref["grads"][name], ref["aref"][name], ref["slack"][name],
                      aref_plain=ref.get("aref_plain", {}).get(name), case=case, **kw)
