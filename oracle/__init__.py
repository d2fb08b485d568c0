"""FP64 CPU oracle for the Gaussian rasterization hot path (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It shares no code with the HIP library
(``paper_2312_10070_amd``) and never imports it.

The native part (``gsr_oracle.cpp``, ``cnn_oracle.cpp``, ``ssim_oracle.cpp``) is plain C++17 in
double precision; :func:`build` compiles it with g++ into ``liboracle.so``
beside the sources. Every function here only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ["gsr_oracle.cpp", "cnn_oracle.cpp", "ssim_oracle.cpp"]
_LIB_PATH = os.environ.get("GSR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

ORC_REC = 24
REC_FIELDS = ["valid", "x", "y", "z_cam", "u", "v", "Sxx", "Sxy", "Syy", "a", "b", "c", "z", "o",
              "px0", "px1", "py0", "py1", "tx0", "tx1", "ty0", "ty1", "margin", "smax"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no fast-math, no FMA contraction)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
           "-o", tmp] + srcs
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.orc_project.argtypes = [i64] + [P] * 9
    lib.orc_render.argtypes = [i64] + [P] * 8 + [ctypes.c_int, i64, P, ctypes.c_int] + [P] * 10
    lib.orc_backward.argtypes = [i64] + [P] * 8 + [ctypes.c_int, i64, P, ctypes.c_int] + [P] * 8
    lib.orc_backward.restype = i64
    lib.orc_tile_lists.argtypes = [i64] + [P] * 8 + [P, P, P, P, i64]
    lib.orc_loss_l1.argtypes = [i64, P, P, P, P, ctypes.c_double, ctypes.c_double, P, P, P]
    lib.orc_loss_reg.argtypes = [i64, P, P, P]
    lib.orc_loss_track.argtypes = [i64, P, P, P, P, P, ctypes.c_double, ctypes.c_float, P, P, P, P, P]
    lib.orc_adam.argtypes = [i64, P, P, P, P, i64] + [ctypes.c_double] * 4
    lib.orc_pose_const_velocity.argtypes = [P, P, P]
    lib.orc_pose_apply_twist.argtypes = [P, P, P]
    if hasattr(lib, "orc_conv2d_fwd"):
        _bind_cnn(lib)
    if hasattr(lib, "orc_ssim"):
        lib.orc_ssim.argtypes = [ctypes.c_int] * 3 + [P] * 5
    _lib = lib
    return lib


def _bind_cnn(lib):
    P = ctypes.c_void_p
    i = ctypes.c_int
    lib.orc_conv2d_fwd.argtypes = [i, i, i, i, i, i, i, i, P, P, P, P]
    lib.orc_conv2d_bwd.argtypes = [i, i, i, i, i, i, i, i, P, P, P, P, P, P]


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    near_z: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def packed(self) -> np.ndarray:
        return _d([self.width, self.height, self.fx, self.fy, self.cx, self.cy, self.near_z, *self.bg])


@dataclass
class Opts:
    lowpass: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    guard: float = 1.3
    tile_w: int = 16
    tile_h: int = 16
    amb_rel: float = 1e-5
    amb_z: float = 1e-6

    def packed(self) -> np.ndarray:
        return _d([self.lowpass, self.alpha_min, self.alpha_max, self.T_min, self.guard, self.tile_w,
                   self.tile_h, self.amb_rel, self.amb_z])


def _params(g):
    """(means, scales, quats, opacities, colors) as contiguous float64 arrays."""
    return [_d(g[k]) for k in ("means", "scales", "quats", "opacities", "colors")]


def project(g: dict, pose7, cam: Camera, opts: Opts) -> dict:
    """Per-Gaussian projection record (O2/O3) as a dict of arrays."""
    lib = _load()
    m, s, q, o, c = _params(g)
    n = m.shape[0]
    out = np.zeros((n, ORC_REC), np.float64)
    lib.orc_project(n, _p(m), _p(s), _p(q), _p(o), _p(c), _p(_d(pose7)), _p(cam.packed()),
                    _p(opts.packed()), _p(out))
    rec = {name: out[:, i] for i, name in enumerate(REC_FIELDS)}
    rec["valid"] = rec["valid"] > 0.5
    return rec


def render(g: dict, pose7, cam: Camera, opts: Opts, mode: int = 1, pixels=None, nthreads: int | None = None):
    """Brute-force FP64 render; returns dict of color [3,H,W], depth, alpha, T, ncomp, amb, alt_*."""
    lib = _load()
    m, s, q, o, c = _params(g)
    n = m.shape[0]
    H, W = cam.height, cam.width
    P = H * W
    color = np.zeros((3, H, W)); depth = np.zeros((H, W)); alpha = np.zeros((H, W))
    T = np.ones((H, W)); ncomp = np.zeros((H, W), np.int32); amb = np.zeros((H, W), np.int32)
    ac = np.zeros((3, H, W)); ad = np.zeros((H, W)); aa = np.zeros((H, W))
    hsh = np.zeros((H, W), np.uint64)
    pix = None if pixels is None else np.ascontiguousarray(np.asarray(pixels, np.int64))
    npix = 0 if pix is None else pix.shape[0]
    nt = nthreads or os.cpu_count() or 1
    lib.orc_render(n, _p(m), _p(s), _p(q), _p(o), _p(c), _p(_d(pose7)), _p(cam.packed()), _p(opts.packed()),
                   mode, npix, _p(pix), nt, _p(color), _p(depth), _p(alpha), _p(T), _p(ncomp), _p(amb),
                   _p(ac), _p(ad), _p(aa), _p(hsh))
    return dict(color=color, depth=depth, alpha=alpha, T=T, ncomp=ncomp, amb=amb, alt_color=ac,
                alt_depth=ad, alt_alpha=aa, hash=hsh)


def split_flat(flat: np.ndarray, n: int) -> dict:
    o = 0
    out = {}
    for name, shape in (("means", (n, 3)), ("scales", (n, 3)), ("quats", (n, 4)), ("opacities", (n,)),
                        ("colors", (n, 3)), ("pose7", (7,)), ("twist6", (6,))):
        size = int(np.prod(shape))
        out[name] = flat[o:o + size].reshape(shape)
        o += size
    return out


def backward(g: dict, pose7, cam: Camera, opts: Opts, gC, gD, gA=None, mode: int = 1, pixels=None,
             nthreads: int | None = None, with_g2d: bool = False) -> dict:
    """Analytic FP64 backward; returns grads, aref, aref_plain, slack (dicts) and n_unverifiable.
    aref: per element, the summed magnitudes of its per-pixel terms (before cancellation), each pixel's
    scaled by that pixel's transmittance condition number kappa; aref_plain: the same without kappa."""
    lib = _load()
    m, s, q, o, c = _params(g)
    n = m.shape[0]
    total = 14 * n + 13
    gflat = np.zeros(total); aref = np.zeros(total); slack = np.zeros(total); aplain = np.zeros(total)
    g2d = np.zeros((n, 10)) if with_g2d else None
    pix = None if pixels is None else np.ascontiguousarray(np.asarray(pixels, np.int64))
    npix = 0 if pix is None else pix.shape[0]
    nt = nthreads or os.cpu_count() or 1
    gCd = _d(gC); gDd = _d(gD); gAd = None if gA is None else _d(gA)
    nu = lib.orc_backward(n, _p(m), _p(s), _p(q), _p(o), _p(c), _p(_d(pose7)), _p(cam.packed()),
                          _p(opts.packed()), mode, npix, _p(pix), nt, _p(gCd), _p(gDd), _p(gAd), _p(gflat),
                          _p(aref), _p(slack), _p(g2d), _p(aplain))
    out = dict(grads=split_flat(gflat, n), aref=split_flat(aref, n), aref_plain=split_flat(aplain, n),
               slack=split_flat(slack, n), n_unverifiable=int(nu))
    if with_g2d:
        out["g2d"] = g2d
    return out


def tile_lists(g: dict, pose7, cam: Camera, opts: Opts) -> dict:
    """Per-tile depth-ordered Gaussian id lists (O6)."""
    lib = _load()
    m, s, q, o, c = _params(g)
    n = m.shape[0]
    ntx = -(-cam.width // opts.tile_w)
    nty = -(-cam.height // opts.tile_h)
    K = np.zeros(1, np.int64)
    counts = np.zeros(n, np.int64)
    ranges = np.zeros((ntx * nty, 2), np.int64)
    args = [n, _p(m), _p(s), _p(q), _p(o), _p(c), _p(_d(pose7)), _p(cam.packed()), _p(opts.packed())]
    lib.orc_tile_lists(*args, _p(K), _p(counts), _p(ranges), None, 0)
    ids = np.zeros(max(int(K[0]), 1), np.int32)
    rc = lib.orc_tile_lists(*args, _p(K), None, None, _p(ids), ids.shape[0])
    assert rc == 0
    return dict(K=int(K[0]), counts=counts, ranges=ranges, ids=ids[:int(K[0])], n_tiles_x=ntx, n_tiles_y=nty)


def loss_l1(C, D, Ct, Dt, w_color=1.0, w_depth=1.0):
    lib = _load()
    C = np.ascontiguousarray(C, np.float32); D = np.ascontiguousarray(D, np.float32)
    Ct = np.ascontiguousarray(Ct, np.float32); Dt = np.ascontiguousarray(Dt, np.float32)
    P = D.size
    loss = np.zeros(1); gC = np.zeros(C.shape); gD = np.zeros(D.shape)
    lib.orc_loss_l1(P, _p(C), _p(D), _p(Ct), _p(Dt), w_color, w_depth, _p(loss), _p(gC), _p(gD))
    return float(loss[0]), gC, gD


def _quat_R(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return q, np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def submap_trigger(pose_first7, pose_cur7, d_thre=0.5, theta_thre=np.deg2rad(50.0)) -> bool:
    """Sub-map creation rule (Sec. 3.2): the camera centres (c = -R^T t of the
    world-to-camera poses) more than d_thre apart, or the relative rotation's
    angle above theta_thre (radians)."""
    qa, Ra = _quat_R(np.asarray(pose_first7, np.float64)[:4])
    qb, Rb = _quat_R(np.asarray(pose_cur7, np.float64)[:4])
    ca = -Ra.T @ np.asarray(pose_first7, np.float64)[4:7]
    cb = -Rb.T @ np.asarray(pose_cur7, np.float64)[4:7]
    angle = 2.0 * np.arccos(min(1.0, abs(float(qa @ qb))))
    return bool(np.linalg.norm(ca - cb) > d_thre or angle > theta_thre)


def compact(groups, keep):
    """Stable compaction: the rows with keep != 0 of every array of every group."""
    k = np.asarray(keep) != 0
    return int(k.sum()), [{n: np.asarray(v)[k] for n, v in g.items()} for g in groups]


def merge_submap(global_params: dict, sub_params: dict, rho: float = 0.01) -> dict:
    """The supplement's merge of a sub-map into the global map: its Gaussians
    with no global mean within rho (the seeding rule) are appended."""
    _, keep = seed_query(global_params["means"], sub_params["means"], rho, rho)
    _, (kept,) = compact([sub_params], keep)
    return {k: np.concatenate([np.asarray(global_params[k]), kept[k]]) for k in global_params}


def seed_candidates(color, depth, alpha, u, pose7, cam: Camera, p_uniform: float, p_grad: float = 0.0,
                    grad_thre: float = 0.0, alpha_n: float = 0.6):
    """Candidate points for new Gaussians (Sec. 3.2 with the supplement's alpha_n).
    A pixel needs a positive observed depth. For a sub-map's first keyframe
    (alpha None) it is chosen iff u < p_uniform + p_grad * [edge], where edge
    means the grey image's central-difference gradient exceeds grad_thre
    (gx^2 + gy^2 > grad_thre^2; grey = ((r + g) + b) / 3; border pixels have no
    gradient); for later keyframes iff alpha < alpha_n and u < p_uniform. The
    random numbers u are inputs. These decisions are taken in binary32 (the
    precision of the images). A chosen pixel (x, y) with depth d back-projects to
    X_c = ((x - cx) d / fx, (y - cy) d / fy, d) and X_w = R^T (X_c - t) for the
    world-to-camera pose (q normalised, t), in FP64. Returns (points [m,3],
    colours [m,3]) in row-major pixel order."""
    f = np.float32
    C = np.asarray(color, f); D = np.asarray(depth, f); U = np.asarray(u, f)
    H, W = D.shape
    gray = ((C[0] + C[1]) + C[2]) / f(3)
    gx = np.zeros((H, W), f); gy = np.zeros((H, W), f)
    gx[1:-1, 1:-1] = gray[1:-1, 2:] - gray[1:-1, :-2]
    gy[1:-1, 1:-1] = gray[2:, 1:-1] - gray[:-2, 1:-1]
    edge = (gx * gx + gy * gy) > f(grad_thre) * f(grad_thre)
    if alpha is None:
        pick = (D > 0) & (U < np.where(edge, f(p_uniform) + f(p_grad), f(p_uniform)))
    else:
        pick = (D > 0) & (np.asarray(alpha, f) < f(alpha_n)) & (U < f(p_uniform))
    ys, xs = np.nonzero(pick)
    d = D[ys, xs].astype(np.float64)
    Xc = np.stack([(xs - cam.cx) * d / cam.fx, (ys - cam.cy) * d / cam.fy, d], 1)
    q = np.asarray(pose7[:4], np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    Xw = (Xc - np.asarray(pose7[4:7], np.float64)) @ R  # rows: R^T (X_c - t)
    return Xw, C[:, ys, xs].T.astype(np.float64)


def seed_query(means, points, rho: float, r_max: float, chunk: int = 128):
    """Neighbour queries of the seeding step (Sec. 3.2 radius test, the
    supplement's nearest-neighbour scale), by brute force over every mean:
    nn_d2[j] = min(r_max^2, min_i d2(q_j, p_i)) with d2 = (dx^2 + dy^2) + dz^2
    in binary32 (the precision of the stored coordinates; numpy does not fuse),
    keep[j] = nn_d2[j] >= rho^2. Returns (nn_d2 float32 [m], keep int32 [m])."""
    p = np.asarray(means, np.float32).reshape(-1, 3)
    q = np.asarray(points, np.float32).reshape(-1, 3)
    r2max = np.float32(r_max) * np.float32(r_max)
    rho2 = np.float32(rho) * np.float32(rho)
    nn = np.full(q.shape[0], r2max, np.float32)
    if p.shape[0] > 0:
        for s in range(0, q.shape[0], chunk):
            qq = q[s:s + chunk]
            dx = qq[:, None, 0] - p[None, :, 0]
            dy = qq[:, None, 1] - p[None, :, 1]
            dz = qq[:, None, 2] - p[None, :, 2]
            d2 = (dx * dx + dy * dy) + dz * dz
            nn[s:s + chunk] = np.minimum(r2max, d2.min(axis=1))
    return nn, (nn >= rho2).astype(np.int32)


def seed_gaussians(points, colors, nn_d2, keep) -> dict:
    """New Gaussians from the seeding step (Sec. 3.2: the sampled points with
    no sub-map Gaussian within rho are added; supplement: opacity 0.5, scale =
    the nearest-neighbour distance in the active sub-map). Every kept point j,
    in order, gives mean = points[j], colour = colors[j], scale = sqrt(nn_d2[j])
    on all three axes (binary32, the precision of the stored distance),
    rotation = identity quaternion (1, 0, 0, 0), opacity 0.5."""
    idx = np.flatnonzero(np.asarray(keep) != 0)
    d = np.sqrt(np.asarray(nn_d2, np.float32)[idx])
    k = idx.shape[0]
    quats = np.zeros((k, 4), np.float32)
    quats[:, 0] = 1.0
    return dict(means=np.asarray(points, np.float32).reshape(-1, 3)[idx],
                scales=np.repeat(d[:, None], 3, axis=1).astype(np.float32),
                quats=quats, opacities=np.full(k, 0.5, np.float32),
                colors=np.asarray(colors, np.float32).reshape(-1, 3)[idx])


def prune(groups, o_thre: float):
    """Opacity pruning (supplement, mapping): Gaussian i is kept iff its opacity
    >= o_thre (NaN is not), and the kept rows stay in their order. groups: a
    list of dicts of arrays with N rows, the first holding "opacities"; the
    decision is taken in binary32, the precision the opacities are stored in.
    Returns (n_kept, [dict of kept rows per group])."""
    o = np.asarray(groups[0]["opacities"], np.float32)
    keep = o >= np.float32(o_thre)
    return int(keep.sum()), [{k: np.asarray(v)[keep] for k, v in g.items()} for g in groups]


def loss_reg(scales):
    """Eq. 11 on [N,3] scales: (L_reg, dL_reg/dscales [N,3])."""
    lib = _load()
    s = _d(scales)
    assert s.ndim == 2 and s.shape[1] == 3
    loss = np.zeros(1); g = np.zeros(s.shape)
    lib.orc_loss_reg(s.shape[0], _p(s), _p(loss), _p(g))
    return float(loss[0]), g


def loss_track(C, D, A, Ct, Dt, lambda_c=0.5, inlier_mult=50.0):
    lib = _load()
    C = np.ascontiguousarray(C, np.float32); D = np.ascontiguousarray(D, np.float32)
    A = np.ascontiguousarray(A, np.float32)
    Ct = np.ascontiguousarray(Ct, np.float32); Dt = np.ascontiguousarray(Dt, np.float32)
    P = D.size
    loss = np.zeros(1); gC = np.zeros(C.shape); gD = np.zeros(D.shape)
    med = np.zeros(1, np.float32); ni = np.zeros(1, np.int64)
    lib.orc_loss_track(P, _p(C), _p(D), _p(A), _p(Ct), _p(Dt), lambda_c, inlier_mult, _p(loss), _p(gC),
                       _p(gD), _p(med), _p(ni))
    return dict(loss=float(loss[0]), gC=gC, gD=gD, median=float(med[0]), n_inlier=int(ni[0]))


def ssim(X, Y, want_grad: bool = True):
    """SSIM(X, Y) of Eq. 10 (Wang et al.'s 11x11 Gaussian window, sigma 1.5,
    zero padding, C1 = 1e-4, C2 = 9e-4) on [C, H, W] images.
    Returns (mean, map[C,H,W], d mean / d X or None)."""
    lib = _load()
    X = _d(X); Y = _d(Y)
    assert X.shape == Y.shape and X.ndim == 3
    Cc, Hh, Ww = X.shape
    mp = np.zeros(X.shape); mean = np.zeros(1)
    g = np.zeros(X.shape) if want_grad else None
    rc = lib.orc_ssim(Cc, Hh, Ww, _p(X), _p(Y), _p(mp), _p(mean), _p(g))
    assert rc == 0
    return float(mean[0]), mp, g


def adam(param, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    lib = _load()
    for a in (param, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    gd = _d(g)
    lib.orc_adam(param.size, _p(param), _p(m), _p(v), _p(gd), step, lr, b1, b2, eps)


def pose_const_velocity(pose_prev2, pose_prev1) -> np.ndarray:
    """Eq. 13 on pose7 = (q, t)."""
    lib = _load()
    a = _d(pose_prev2); b = _d(pose_prev1); out = np.zeros(7)
    lib.orc_pose_const_velocity(_p(a), _p(b), _p(out))
    return out


# ---------------------------------------------------------------------------
# CNN oracle (tracking-initialisation network), FP64, NCHW
# ---------------------------------------------------------------------------

def conv2d(x, w, b, stride=2, pad=1):
    """3x3 (k x k) convolution by definition; x [B,C,H,W], w [O,C,k,k], b [O] or None."""
    lib = _load()
    x = _d(x); w = _d(w)
    B, C, H, W = x.shape
    O, _, k, _ = w.shape
    oh = (H + 2 * pad - k) // stride + 1
    ow = (W + 2 * pad - k) // stride + 1
    out = np.zeros((B, O, oh, ow))
    bb = None if b is None else _d(b)
    lib.orc_conv2d_fwd(B, C, H, W, O, stride, pad, k, _p(x), _p(w), _p(bb), _p(out))
    return out


def conv2d_bwd(x, w, dout, stride=2, pad=1, want_dx=True):
    """(dx or None, dw, db) of conv2d for upstream dout."""
    lib = _load()
    x = _d(x); w = _d(w); dout = _d(dout)
    B, C, H, W = x.shape
    O, _, k, _ = w.shape
    dx = np.zeros_like(x) if want_dx else None
    dw = np.zeros_like(w)
    db = np.zeros(O)
    lib.orc_conv2d_bwd(B, C, H, W, O, stride, pad, k, _p(x), _p(w), _p(dout), _p(dx), _p(dw), _p(db))
    return dx, dw, db


def moment_basis(h: int, w: int) -> np.ndarray:
    """[3, h, w]: 1, x^ and y^ at the pixel centres, x^ = (2 x + 1) / w - 1,
    y^ = (2 y + 1) / h - 1 (both in (-1, 1))."""
    xs = (2.0 * np.arange(w) + 1.0) / w - 1.0
    ys = (2.0 * np.arange(h) + 1.0) / h - 1.0
    return np.stack([np.ones((h, w)), np.broadcast_to(xs[None, :], (h, w)), np.broadcast_to(ys[:, None], (h, w))])


def initnet_forward(x, params):
    """x [B,8,H,W]; params: w0..w3 [64,C,3,3], b0..b3 [64], wfc [6,3C], bfc [6].
    Four stride-2 3x3 convolutions with ReLU, moment pooling (per channel the
    mean of the last map and its means weighted by x^ and y^, k-major:
    pool[b, 64 k + c]), linear head. Returns (out [B,6], cache)."""
    acts = [np.asarray(x, np.float64)]
    for l in range(4):
        y = conv2d(acts[-1], params[f"w{l}"], params[f"b{l}"])
        acts.append(np.maximum(y, 0.0))
    a = acts[-1]
    basis = moment_basis(a.shape[2], a.shape[3])
    pool = np.einsum("bchw,khw->bkc", a, basis).reshape(a.shape[0], -1) / (a.shape[2] * a.shape[3])
    out = pool @ np.asarray(params["wfc"], np.float64).T + np.asarray(params["bfc"], np.float64)
    return out, (acts, pool)


def initnet_backward(params, cache, dout):
    """Gradients of the network parameters for upstream dL/dout [B,6]."""
    acts, pool = cache
    grads = {"wfc": dout.T @ pool, "bfc": dout.sum(0)}
    a = acts[-1]
    B, C, h, w = a.shape
    dpool = (dout @ np.asarray(params["wfc"], np.float64)).reshape(B, 3, C)
    dact = np.einsum("bkc,khw->bchw", dpool, moment_basis(h, w)) / (h * w)
    for l in range(3, -1, -1):
        dy = dact * (acts[l + 1] > 0)
        dx, dw, db = conv2d_bwd(acts[l], params[f"w{l}"], dy, want_dx=l > 0)
        grads[f"w{l}"] = dw
        grads[f"b{l}"] = db
        dact = dx
    return grads


def initnet_loss(out, label, scale):
    """L = 1/(2B) sum_b sum_j ((out - label) / scale_j)^2 and dL/dout."""
    r = (np.asarray(out, np.float64) - np.asarray(label, np.float64)) / np.asarray(scale, np.float64)
    B = r.shape[0]
    return 0.5 * float((r * r).sum()) / B, r / np.asarray(scale, np.float64) / B


def pose_apply_twist(pose7, twist6) -> np.ndarray:
    """exp(xi^) T (Rodrigues), unit quaternion with w >= 0."""
    lib = _load()
    a = _d(pose7); x = _d(twist6); out = np.zeros(7)
    lib.orc_pose_apply_twist(_p(a), _p(x), _p(out))
    return out
