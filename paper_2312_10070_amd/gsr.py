"""ctypes binding of libgsr.so (the C ABI in include/gsr.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the rendering path runs in the library's kernels. The
library is loaded from this package directory; if it is missing, or no HIP
device is present, calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsr.so")

GSR_OK, GSR_EINVAL, GSR_ENOMEM, GSR_EHIP, GSR_EOVERFLOW = 0, -1, -2, -3, -4


class GsrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libgsr error {code}: {msg}")
        self.code = code


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("near_z", ctypes.c_float), ("bg", ctypes.c_float * 3)]


class Opts(ctypes.Structure):
    _fields_ = [("lowpass", ctypes.c_float), ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("T_min", ctypes.c_float), ("guard", ctypes.c_float), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("deterministic", ctypes.c_int32)]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacities", ctypes.c_void_p), ("colors", ctypes.c_void_p)]


class Grads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacities", ctypes.c_void_p), ("colors", ctypes.c_void_p)]


class Adam5(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p * 5), ("exp_avg", ctypes.c_void_p * 5), ("exp_avg_sq", ctypes.c_void_p * 5),
                ("lr", ctypes.c_float * 5), ("step", ctypes.c_int64), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("scale_reg", ctypes.c_float)]


class TrackOpts(ctypes.Structure):
    _fields_ = [("lambda_c", ctypes.c_float), ("inlier_mult", ctypes.c_float), ("lr_q", ctypes.c_float),
                ("lr_t", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("n_iters", ctypes.c_int32)]


_lib = None
_lock = threading.Lock()

# name -> (restype, argtypes)
P = ctypes.c_void_p
_SIGS = {
    "gsr_ctx_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, P]),
    "gsr_ctx_destroy": (ctypes.c_int, [P]),
    "gsr_set_stream": (ctypes.c_int, [P, P]),
    "gsr_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "gsr_last_error": (ctypes.c_char_p, [P]),
    "gsr_default_opts": (None, [ctypes.POINTER(Opts)]),
    "gsr_render_fwd": (ctypes.c_int, [P, ctypes.POINTER(Gaussians), ctypes.POINTER(Camera), ctypes.POINTER(Opts), P,
                                      P, P, P, ctypes.POINTER(P)]),
    "gsr_render_bwd": (ctypes.c_int, [P, P, P, P, P, ctypes.POINTER(Grads), P, P]),
    "gsr_render_bwd_adam": (ctypes.c_int, [P, P, P, P, P, ctypes.POINTER(Adam5)]),
    "gsr_render_fwd_batch": (ctypes.c_int, [P, ctypes.POINTER(Gaussians), ctypes.c_int32, ctypes.POINTER(Camera),
                                            ctypes.POINTER(Opts), ctypes.c_int32, P, P, P, P, ctypes.POINTER(P)]),
    "gsr_autotune_batch": (ctypes.c_int, [P, ctypes.POINTER(Gaussians), ctypes.c_int32, ctypes.POINTER(Camera),
                                          ctypes.POINTER(Opts), P, P, P, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32), P]),
    "gsr_state_release": (ctypes.c_int, [P, P]),
    "gsr_tile_lists": (ctypes.c_int, [P, P, ctypes.POINTER(ctypes.c_int64), P, P]),
    "gsr_loss_l1": (ctypes.c_int, [P, P, P, P, P, ctypes.c_int64, ctypes.c_float, ctypes.c_float, P, P, P]),
    "gsr_loss_reg": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_float, P, P]),
    "gsr_seed_candidates": (ctypes.c_int, [P, ctypes.POINTER(Camera), P, P, P, P, P, ctypes.c_float, ctypes.c_float,
                                           ctypes.c_float, ctypes.c_float, P, P, ctypes.POINTER(ctypes.c_int64)]),
    "gsr_seed_query": (ctypes.c_int, [P, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_float, ctypes.c_float, P, P]),
    "gsr_compact": (ctypes.c_int, [P, ctypes.c_int64, P, P, P, ctypes.POINTER(ctypes.c_int64)]),
    "gsr_seed_gaussians": (ctypes.c_int, [P, ctypes.c_int64, P, P, P, P, P, ctypes.POINTER(ctypes.c_int64)]),
    "gsr_submap_offload": (ctypes.c_int, [P, ctypes.c_int64, P, P]),
    "gsr_submap_restore": (ctypes.c_int, [P, ctypes.c_int64, P, P]),
    "gsr_submap_trigger": (ctypes.c_int, [P, P, ctypes.c_float, ctypes.c_float, ctypes.POINTER(ctypes.c_int32)]),
    "gsr_prune": (ctypes.c_int, [P, ctypes.c_int64, ctypes.c_float, P, P, ctypes.POINTER(ctypes.c_int64)]),
    "gsr_loss_ssim": (ctypes.c_int, [P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, P, P]),
    "gsr_loss_track": (ctypes.c_int, [P, P, P, P, P, P, ctypes.c_int64, ctypes.c_float, ctypes.c_float, P, P, P, P]),
    "gsr_loss_track_noalloc": (ctypes.c_int, [P, P, P, P, P, P, ctypes.c_int64, ctypes.c_float, ctypes.c_float, P, P,
                                              P, P]),
    "gsr_adam": (ctypes.c_int, [P, P, P, P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float]),
    "gsr_adam_groups": (ctypes.c_int, [P, ctypes.c_int32, P, P, P, P, P, P, ctypes.c_int64, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float]),
    "gsr_pose_const_velocity": (ctypes.c_int, [P, P, P, P]),
    "gsr_pose_adam": (ctypes.c_int, [P, P, P, P] + [ctypes.c_float] * 5),
    "gsr_pose_apply_twist": (ctypes.c_int, [P, P, P, P]),
    "gsr_track_graph_create": (ctypes.c_int, [P, ctypes.POINTER(Gaussians), ctypes.POINTER(Camera),
                                              ctypes.POINTER(Opts), ctypes.POINTER(TrackOpts), P, P, ctypes.c_int64,
                                              ctypes.POINTER(P)]),
    "gsr_track_graph_set_frame": (ctypes.c_int, [P, P, P, P]),
    "gsr_track_graph_run": (ctypes.c_int, [P, P, P, P]),
    "gsr_track_graph_destroy": (ctypes.c_int, [P, P]),
    "gsr_initnet_create": (ctypes.c_int, [P, ctypes.c_int32, ctypes.POINTER(P)]),
    "gsr_initnet_destroy": (ctypes.c_int, [P, P]),
    "gsr_initnet_count": (ctypes.c_int, [P, P, ctypes.POINTER(ctypes.c_int64)]),
    "gsr_initnet_set_params": (ctypes.c_int, [P, P, P]),
    "gsr_initnet_get_params": (ctypes.c_int, [P, P, P, P]),
    "gsr_initnet_set_input": (ctypes.c_int, [P, P, ctypes.c_int32, P]),
    "gsr_initnet_get_activation": (ctypes.c_int, [P, P, ctypes.c_int32, ctypes.c_int32, P, P]),
    "gsr_pack_rgbd_pair": (ctypes.c_int, [P, P, P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, P]),
    "gsr_initnet_forward": (ctypes.c_int, [P, P, ctypes.c_int32, P]),
    "gsr_initnet_backward": (ctypes.c_int, [P, P, ctypes.c_int32, P, P, P, P]),
    "gsr_initnet_adam": (ctypes.c_int, [P, P] + [ctypes.c_float] * 4),
    "gsr_profile_enable": (ctypes.c_int, [P, ctypes.c_int]),
    "gsr_profile_only": (ctypes.c_int, [P, ctypes.c_char_p]),
    "gsr_profile_read": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_char_p, P, P, ctypes.POINTER(ctypes.c_int)]),
    "gsr_state_stats": (ctypes.c_int, [P, P, P]),
}
OPTIONAL_SIGS = {}


def declared_symbols() -> list[str]:
    return list(_SIGS) + list(OPTIONAL_SIGS)


def load(path: str = LIB_PATH):
    """Load libgsr.so (without touching the GPU) and bind its signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise FileNotFoundError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; "
                                    f"g.build()'` (hipcc, gfx950)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in {**_SIGS, **OPTIONAL_SIGS}.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libgsr takes device tensors only")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t, name, shape=None):
    if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    return t


@dataclass
class RasterOpts:
    lowpass: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    guard: float = 1.3
    tile_w: int = 16
    tile_h: int = 16
    deterministic: int = 0  # 1: bitwise reproducible backward (fixed-order sums, more memory, slower)

    def c(self) -> Opts:
        return Opts(self.lowpass, self.alpha_min, self.alpha_max, self.T_min, self.guard, self.tile_w, self.tile_h,
                    int(self.deterministic))


def make_camera(width, height, fx, fy, cx, cy, near_z=0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    return Camera(int(width), int(height), float(fx), float(fy), float(cx), float(cy), float(near_z),
                  (ctypes.c_float * 3)(*[float(b) for b in bg]))


def camera_from(intr, bg=(0.0, 0.0, 0.0)) -> Camera:
    return make_camera(intr.width, intr.height, intr.fx, intr.fy, intr.cx, intr.cy, intr.near_z, bg)


class Context:
    """One libgsr context per device; enqueues on torch's current stream."""

    _per_device: dict[int, "Context"] = {}

    def __init__(self, device: int = 0):
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("libgsr needs a HIP device; none is available")
        self.lib = lib
        self.device = device
        h = P()
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream(device).cuda_stream
        rc = lib.gsr_ctx_create(ctypes.byref(h), device, P(stream))
        if rc != GSR_OK:
            raise GsrError(rc, lib.gsr_strerror(rc).decode())
        self.h = h

    @classmethod
    def get(cls, device: int = 0) -> "Context":
        if device not in cls._per_device:
            cls._per_device[device] = Context(device)
        return cls._per_device[device]

    def check(self, rc):
        if rc != GSR_OK:
            msg = self.lib.gsr_last_error(self.h).decode()
            raise GsrError(rc, msg)

    def sync_stream(self):
        self.check(self.lib.gsr_set_stream(self.h, P(torch.cuda.current_stream(self.device).cuda_stream)))


class State:
    """Handle of one forward's saved state; released when garbage-collected."""

    def __init__(self, ctx: Context, h, keep):
        self.ctx = ctx
        self.h = h
        self.keep = keep  # tensors the backward re-reads

    def release(self):
        if self.h is not None:
            self.ctx.lib.gsr_state_release(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def _gaussians(means, scales, quats, opacities, colors) -> Gaussians:
    n = means.shape[0]
    _f32(means, "means", (n, 3)); _f32(scales, "scales", (n, 3)); _f32(quats, "quats", (n, 4))
    _f32(opacities, "opacities", (n,)); _f32(colors, "colors", (n, 3))
    if n > 0 and quats.data_ptr() % 16:
        raise ValueError("quats must be 16-byte aligned")
    return Gaussians(n, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opacities), _ptr(colors))


def render_fwd(means, scales, quats, opacities, colors, pose7, camera: Camera, opts: RasterOpts | None = None,
               ctx: Context | None = None):
    """Forward render; returns (color [3,H,W], depth [H,W], alpha [H,W], State)."""
    ctx = ctx or Context.get(means.device.index or 0)
    ctx.sync_stream()
    opts = opts or RasterOpts()
    g = _gaussians(means, scales, quats, opacities, colors)
    _f32(pose7, "pose7", (7,))
    H, W = camera.height, camera.width
    dev = means.device
    color = torch.empty((3, H, W), device=dev, dtype=torch.float32)
    depth = torch.empty((H, W), device=dev, dtype=torch.float32)
    alpha = torch.empty((H, W), device=dev, dtype=torch.float32)
    st = P()
    oc = opts.c()
    ctx.check(ctx.lib.gsr_render_fwd(ctx.h, ctypes.byref(g), ctypes.byref(camera), ctypes.byref(oc), _ptr(pose7),
                                     _ptr(color), _ptr(depth), _ptr(alpha), ctypes.byref(st)))
    state = State(ctx, st, (means, scales, quats, opacities, colors, pose7))
    state.shape = (H, W)
    return color, depth, alpha, state


def render_fwd_batch(means, scales, quats, opacities, colors, poses7, camera: Camera, opts: RasterOpts | None = None,
                     blocks_per_cu: int = 0, ctx: Context | None = None):
    """Batched forward over V views (poses7 [V,7]); returns color [V,3,H,W], depth, alpha [V,H,W], State."""
    ctx = ctx or Context.get(means.device.index or 0)
    ctx.sync_stream()
    opts = opts or RasterOpts()
    g = _gaussians(means, scales, quats, opacities, colors)
    V = poses7.shape[0]
    _f32(poses7, "poses7", (V, 7))
    H, W = camera.height, camera.width
    dev = means.device
    color = torch.empty((V, 3, H, W), device=dev, dtype=torch.float32)
    depth = torch.empty((V, H, W), device=dev, dtype=torch.float32)
    alpha = torch.empty((V, H, W), device=dev, dtype=torch.float32)
    st = P()
    oc = opts.c()
    ctx.check(ctx.lib.gsr_render_fwd_batch(ctx.h, ctypes.byref(g), V, ctypes.byref(camera), ctypes.byref(oc),
                                           int(blocks_per_cu), _ptr(poses7), _ptr(color), _ptr(depth), _ptr(alpha),
                                           ctypes.byref(st)))
    state = State(ctx, st, (means, scales, quats, opacities, colors, poses7))
    state.shape = (H, W)
    state.views = V
    return color, depth, alpha, state


def autotune_batch(means, scales, quats, opacities, colors, poses7, camera: Camera, dL_dcolor, dL_ddepth,
                   opts: RasterOpts | None = None, reps: int = 3, ctx: Context | None = None):
    """Returns (RasterOpts with the fastest tile shape, blocks_per_cu, {(tw, th, bpc): ms})."""
    import numpy as np
    ctx = ctx or Context.get(means.device.index or 0)
    ctx.sync_stream()
    opts = opts or RasterOpts()
    g = _gaussians(means, scales, quats, opacities, colors)
    V = poses7.shape[0]
    oc = opts.c()
    bpc = ctypes.c_int32()
    table = np.zeros(15, np.float32)
    ctx.check(ctx.lib.gsr_autotune_batch(ctx.h, ctypes.byref(g), V, ctypes.byref(camera), ctypes.byref(oc),
                                         _ptr(poses7), _ptr(_f32(dL_dcolor, "dL_dcolor")),
                                         _ptr(_f32(dL_ddepth, "dL_ddepth")), int(reps), ctypes.byref(bpc),
                                         table.ctypes.data_as(P)))
    best = RasterOpts(opts.lowpass, opts.alpha_min, opts.alpha_max, opts.T_min, opts.guard, oc.tile_w, oc.tile_h,
                      opts.deterministic)
    shapes = [(16, 16), (8, 32), (32, 8)]
    bpcs = [0, 1, 2, 4, 8]
    timings = {(shapes[i // 5][0], shapes[i // 5][1], bpcs[i % 5]): float(table[i]) for i in range(15)}
    return best, int(bpc.value), timings


def render_bwd(state: State, dL_dcolor, dL_ddepth, dL_dalpha=None, want_params=True, want_pose=True, groups=None):
    """Backward; returns dict of gradients (means, scales, quats, opacities, colors, pose7, twist6).
    groups: the parameter groups wanted (default: all five when want_params)."""
    ctx = state.ctx
    ctx.sync_stream()
    means, scales, quats, opacities, colors, pose7 = state.keep
    n = means.shape[0]
    dev = means.device
    gC = _f32(dL_dcolor.contiguous(), "dL_dcolor")
    gD = _f32(dL_ddepth.contiguous(), "dL_ddepth")
    gA = None if dL_dalpha is None else _f32(dL_dalpha.contiguous(), "dL_dalpha")
    out = {}
    if want_params:
        wanted = PARAM_GROUPS if groups is None else tuple(groups)
        for k, shape in (("means", (n, 3)), ("scales", (n, 3)), ("quats", (n, 4)), ("opacities", (n,)),
                         ("colors", (n, 3))):
            if k in wanted:
                out[k] = torch.empty(shape, device=dev, dtype=torch.float32)
        gr = Grads(*[_ptr(out.get(k)) for k in ("means", "scales", "quats", "opacities", "colors")])
    else:
        gr = Grads()
    if want_pose:
        V = getattr(state, "views", None)
        out["pose7"] = torch.empty((7,) if V is None else (V, 7), device=dev, dtype=torch.float32)
        out["twist6"] = torch.empty((6,) if V is None else (V, 6), device=dev, dtype=torch.float32)
    ctx.check(ctx.lib.gsr_render_bwd(ctx.h, state.h, _ptr(gC), _ptr(gD), _ptr(gA), ctypes.byref(gr),
                                     _ptr(out.get("pose7")), _ptr(out.get("twist6"))))
    return out


PARAM_GROUPS = ("means", "scales", "quats", "opacities", "colors")


def render_bwd_adam(state: State, dL_dcolor, dL_ddepth, exp_avg: dict, exp_avg_sq: dict, lrs: dict, step: int,
                    dL_dalpha=None, beta1=0.9, beta2=0.999, eps=1e-8, scale_reg=0.0):
    """Backward fused with one Adam step on the five parameter tensors the
    forward read (updated in place, as are the moments; keyed by PARAM_GROUPS).
    scale_reg = lambda_reg adds the Eq. 11 regulariser's gradient to the scales'."""
    ctx = state.ctx
    ctx.sync_stream()
    params = dict(zip(PARAM_GROUPS, state.keep[:5]))
    gC = _f32(dL_dcolor.contiguous(), "dL_dcolor")
    gD = _f32(dL_ddepth.contiguous(), "dL_ddepth")
    gA = None if dL_dalpha is None else _f32(dL_dalpha.contiguous(), "dL_dalpha")
    a = Adam5()
    for i, k in enumerate(PARAM_GROUPS):
        for t, nme in ((exp_avg[k], "exp_avg"), (exp_avg_sq[k], "exp_avg_sq")):
            _f32(t, nme)
            if t.shape != params[k].shape or not t.is_contiguous():
                raise ValueError(f"{nme}[{k}] must be a contiguous tensor shaped like the parameter")
        a.params[i] = _ptr(params[k])
        a.exp_avg[i] = _ptr(exp_avg[k])
        a.exp_avg_sq[i] = _ptr(exp_avg_sq[k])
        a.lr[i] = float(lrs[k])
    a.step = int(step)
    a.beta1, a.beta2, a.eps = float(beta1), float(beta2), float(eps)
    a.scale_reg = float(scale_reg)
    ctx.check(ctx.lib.gsr_render_bwd_adam(ctx.h, state.h, _ptr(gC), _ptr(gD), _ptr(gA), ctypes.byref(a)))


def tile_lists(state: State, n_tiles: int):
    """(K, ranges int32 [n_tiles,2], ids int32 [K]) of a forward (synchronises)."""
    ctx = state.ctx
    ctx.sync_stream()
    K = ctypes.c_int64()
    ctx.check(ctx.lib.gsr_tile_lists(ctx.h, state.h, ctypes.byref(K), None, None))
    dev = state.keep[0].device
    ranges = torch.empty((n_tiles, 2), device=dev, dtype=torch.int32)
    ids = torch.empty((max(K.value, 1),), device=dev, dtype=torch.int32)
    ctx.check(ctx.lib.gsr_tile_lists(ctx.h, state.h, ctypes.byref(K), _ptr(ranges), _ptr(ids)))
    return K.value, ranges, ids[:K.value]


def loss_l1(color, depth, tgt_color, tgt_depth, w_color=1.0, w_depth=1.0, ctx: Context | None = None):
    """Mapping L1 loss; returns (loss [1] device, dL/dcolor, dL/ddepth)."""
    ctx = ctx or Context.get(color.device.index or 0)
    ctx.sync_stream()
    P_ = depth.numel()
    for t, nme in ((color, "color"), (depth, "depth"), (tgt_color, "tgt_color"), (tgt_depth, "tgt_depth")):
        _f32(t, nme)
    loss = torch.empty(1, device=color.device, dtype=torch.float32)
    gC = torch.empty_like(color)
    gD = torch.empty_like(depth)
    ctx.check(ctx.lib.gsr_loss_l1(ctx.h, _ptr(color), _ptr(depth), _ptr(tgt_color), _ptr(tgt_depth), P_,
                                  float(w_color), float(w_depth), _ptr(loss), _ptr(gC), _ptr(gD)))
    return loss, gC, gD


def seed_candidates(color, depth, u, pose7, camera: Camera, p_uniform: float, p_grad: float = 0.0,
                    grad_thre: float = 0.0, alpha=None, alpha_n: float = 0.6, ctx: Context | None = None):
    """Seeding candidates (see gsr_seed_candidates): (points [m,3], colours [m,3])."""
    ctx = ctx or Context.get(depth.device.index or 0)
    ctx.sync_stream()
    H, W = int(camera.height), int(camera.width)
    _f32(color, "color", (3, H, W)); _f32(depth, "depth", (H, W)); _f32(u, "u", (H, W))
    _f32(pose7, "pose7", (7,))
    if alpha is not None:
        _f32(alpha, "alpha", (H, W))
    pts = torch.empty((H * W, 3), device=depth.device, dtype=torch.float32)
    cols = torch.empty((H * W, 3), device=depth.device, dtype=torch.float32)
    n = ctypes.c_int64()
    ctx.check(ctx.lib.gsr_seed_candidates(ctx.h, ctypes.byref(camera), _ptr(pose7), _ptr(color), _ptr(depth),
                                          _ptr(alpha), _ptr(u), float(p_uniform), float(p_grad), float(grad_thre),
                                          float(alpha_n), _ptr(pts), _ptr(cols), ctypes.byref(n)))
    return pts[:n.value], cols[:n.value]


def seed_query(means, points, rho: float, r_max: float, ctx: Context | None = None):
    """Seeding neighbour queries: (nn_d2 [m] float32, keep [m] int32) of the
    query points [m,3] against the sub-map means [n,3] (see gsr_seed_query)."""
    ctx = ctx or Context.get(points.device.index or 0)
    ctx.sync_stream()
    for t, nme in ((means, "means"), (points, "points")):
        _f32(t, nme)
        if t.dim() != 2 or t.shape[1] != 3:
            raise ValueError(f"{nme} must be [k, 3]")
    m = points.shape[0]
    nn = torch.empty(m, device=points.device, dtype=torch.float32)
    keep = torch.empty(m, device=points.device, dtype=torch.int32)
    ctx.check(ctx.lib.gsr_seed_query(ctx.h, _ptr(means), int(means.shape[0]), _ptr(points), m, float(rho),
                                     float(r_max), _ptr(nn), _ptr(keep)))
    return nn, keep


def seed_gaussians(points, colors, nn_d2, keep, ctx: Context | None = None) -> dict:
    """New Gaussians from the kept seeding points (see gsr_seed_gaussians):
    {means, scales, quats, opacities, colors} with one row per kept point."""
    ctx = ctx or Context.get(points.device.index or 0)
    ctx.sync_stream()
    m = points.shape[0]
    _f32(points, "points", (m, 3)); _f32(colors, "colors", (m, 3)); _f32(nn_d2, "nn_d2", (m,))
    if keep.dtype != torch.int32 or keep.shape != (m,) or not keep.is_contiguous():
        raise ValueError("keep must be a contiguous int32 [m] tensor")
    dev = points.device
    out = {k: torch.empty((m,) + sh, device=dev, dtype=torch.float32)
           for k, sh in (("means", (3,)), ("scales", (3,)), ("quats", (4,)), ("opacities", ()), ("colors", (3,)))}
    arr = (P * 5)(*[P(out[k].data_ptr()) for k in ("means", "scales", "quats", "opacities", "colors")])
    n_new = ctypes.c_int64()
    ctx.check(ctx.lib.gsr_seed_gaussians(ctx.h, m, _ptr(points), _ptr(colors), _ptr(nn_d2), _ptr(keep), arr,
                                         ctypes.byref(n_new)))
    return {k: v[:n_new.value] for k, v in out.items()}


def _compact_call(params, exp_avg, exp_avg_sq, call):
    groups = [params, exp_avg, exp_avg_sq]
    ins = (P * 15)()
    outs = (P * 15)()
    res = [None, None, None]
    for gi, grp in enumerate(groups):
        if grp is None:
            continue
        res[gi] = {}
        for i, k in enumerate(PARAM_GROUPS):
            t = _f32(grp[k], k, tuple(params[k].shape))
            o = torch.empty_like(t)
            ins[5 * gi + i] = _ptr(t)
            outs[5 * gi + i] = _ptr(o)
            res[gi][k] = o
    kept = ctypes.c_int64()
    call(ins, outs, ctypes.byref(kept))
    m = kept.value
    res = [None if r is None else {k: v[:m] for k, v in r.items()} for r in res]
    return m, res[0], res[1], res[2]


def compact(params: dict, keep, exp_avg: dict | None = None, exp_avg_sq: dict | None = None,
            ctx: Context | None = None):
    """Stable compaction of the Gaussians with keep != 0 (int32 [n] device);
    returns (n_kept, params, exp_avg, exp_avg_sq) as new tensors."""
    ctx = ctx or Context.get(params["means"].device.index or 0)
    ctx.sync_stream()
    n = params["opacities"].shape[0]
    if keep.dtype != torch.int32 or not keep.is_cuda or not keep.is_contiguous() or keep.shape != (n,):
        raise ValueError("keep must be a contiguous int32 device tensor of n entries")
    return _compact_call(params, exp_avg, exp_avg_sq,
                         lambda i, o, k: ctx.check(ctx.lib.gsr_compact(ctx.h, n, _ptr(keep), i, o, k)))


def merge_submap(global_params: dict, sub_params: dict, rho: float = 0.01, ctx: Context | None = None):
    """The supplement's merge: the sub-map's Gaussians with no global-map mean
    within rho are appended to the global map; returns the merged parameters."""
    _, keep = seed_query(global_params["means"], sub_params["means"], rho, rho, ctx=ctx)
    _, kept, _, _ = compact(sub_params, keep, ctx=ctx)
    return {k: torch.cat([global_params[k], kept[k]]) for k in PARAM_GROUPS}


def offload_submap(params: dict, ctx: Context | None = None):
    """Copies a finished sub-map's parameters (PARAM_GROUPS, device) into one
    pinned host tensor of 14 n floats [means | scales | quats | opacities |
    colors] (gsr_submap_offload); the copy is enqueued on the current stream
    and complete once that stream is synchronised."""
    ctx = ctx or Context.get(params["means"].device.index or 0)
    ctx.sync_stream()
    n = params["opacities"].shape[0]
    for k, w in zip(PARAM_GROUPS, (3, 3, 4, 1, 3)):
        _f32(params[k], k, (n, w) if w > 1 else (n,))
    host = torch.empty(14 * n, dtype=torch.float32, pin_memory=True)
    arr = (P * 5)(*[params[k].data_ptr() for k in PARAM_GROUPS])
    ctx.check(ctx.lib.gsr_submap_offload(ctx.h, n, arr, ctypes.c_void_p(host.data_ptr())))
    return host


def restore_submap(host, n: int, device=None, ctx: Context | None = None) -> dict:
    """The inverse of offload_submap: new device tensors keyed by PARAM_GROUPS
    (gsr_submap_restore), enqueued on the current stream."""
    device = torch.device(device if device is not None else "cuda")
    ctx = ctx or Context.get(device.index or 0)
    ctx.sync_stream()
    if host.dtype != torch.float32 or host.is_cuda or not host.is_contiguous() or host.numel() != 14 * n:
        raise ValueError("host must be a contiguous float32 CPU tensor of 14 n values")
    out = {k: torch.empty((n, w) if w > 1 else (n,), device=device, dtype=torch.float32)
           for k, w in zip(PARAM_GROUPS, (3, 3, 4, 1, 3))}
    arr = (P * 5)(*[out[k].data_ptr() for k in PARAM_GROUPS])
    ctx.check(ctx.lib.gsr_submap_restore(ctx.h, n, ctypes.c_void_p(host.data_ptr()), arr))
    return out


def submap_trigger(pose_first7, pose_cur7, d_thre: float = 0.5, theta_thre_deg: float = 50.0) -> bool:
    """Sub-map creation rule of Sec. 3.2 (host poses, 7 floats each)."""
    lib = load()
    a = (ctypes.c_float * 7)(*[float(v) for v in pose_first7])
    b = (ctypes.c_float * 7)(*[float(v) for v in pose_cur7])
    out = ctypes.c_int32()
    rc = lib.gsr_submap_trigger(a, b, float(d_thre), float(math.radians(theta_thre_deg)), ctypes.byref(out))
    if rc != GSR_OK:
        raise GsrError(rc, "invalid poses or thresholds")
    return bool(out.value)


def prune(params: dict, o_thre: float, exp_avg: dict | None = None, exp_avg_sq: dict | None = None,
          ctx: Context | None = None):
    """Opacity pruning (stable compaction of the Gaussians with opacity >= o_thre).
    params (and the optional Adam moments) are keyed by PARAM_GROUPS; returns
    (n_kept, params, exp_avg, exp_avg_sq) as new tensors of n_kept rows."""
    ctx = ctx or Context.get(params["means"].device.index or 0)
    ctx.sync_stream()
    n = params["opacities"].shape[0]
    groups = [params, exp_avg, exp_avg_sq]
    ins = (P * 15)()
    outs = (P * 15)()
    res = [None, None, None]
    for gi, grp in enumerate(groups):
        if grp is None:
            continue
        res[gi] = {}
        for i, k in enumerate(PARAM_GROUPS):
            t = _f32(grp[k], k, tuple(params[k].shape))
            o = torch.empty_like(t)
            ins[5 * gi + i] = _ptr(t)
            outs[5 * gi + i] = _ptr(o)
            res[gi][k] = o
    kept = ctypes.c_int64()
    ctx.check(ctx.lib.gsr_prune(ctx.h, n, float(o_thre), ins, outs, ctypes.byref(kept)))
    m = kept.value
    res = [None if r is None else {k: v[:m] for k, v in r.items()} for r in res]
    return m, res[0], res[1], res[2]


def loss_reg(scales, weight, loss, dL_dscales=None, ctx: Context | None = None):
    """Isotropic scale regulariser (Eq. 11), in place: loss [1] += weight L_reg and,
    if given, dL_dscales [n,3] += its gradient."""
    ctx = ctx or Context.get(scales.device.index or 0)
    ctx.sync_stream()
    _f32(scales, "scales")
    _f32(loss, "loss")
    if scales.dim() != 2 or scales.shape[1] != 3 or loss.numel() != 1:
        raise ValueError("scales must be [n, 3] and loss must hold one float")
    if dL_dscales is not None:
        _f32(dL_dscales, "dL_dscales", tuple(scales.shape))
    ctx.check(ctx.lib.gsr_loss_reg(ctx.h, _ptr(scales), int(scales.shape[0]), float(weight), _ptr(loss),
                                   _ptr(dL_dscales)))
    return loss


def loss_ssim(color, tgt_color, weight, loss, dL_dcolor, ctx: Context | None = None):
    """SSIM term of Eq. 10, in place: loss [1] += weight (1 - SSIM(color, tgt_color)),
    dL_dcolor += its gradient. color, tgt_color, dL_dcolor: [3, H, W]."""
    ctx = ctx or Context.get(color.device.index or 0)
    ctx.sync_stream()
    for t, nme in ((color, "color"), (tgt_color, "tgt_color"), (loss, "loss"), (dL_dcolor, "dL_dcolor")):
        _f32(t, nme)
    if color.dim() != 3 or color.shape[0] != 3 or tgt_color.shape != color.shape or dL_dcolor.shape != color.shape:
        raise ValueError("color, tgt_color and dL_dcolor must share one [3, H, W] shape")
    if loss.numel() != 1:
        raise ValueError("loss must hold one float")
    ctx.check(ctx.lib.gsr_loss_ssim(ctx.h, _ptr(color), _ptr(tgt_color), int(color.shape[2]), int(color.shape[1]),
                                    float(weight), _ptr(loss), _ptr(dL_dcolor)))
    return loss, dL_dcolor


def loss_map(color, depth, tgt_color, tgt_depth, lam=0.2, w_color=1.0, w_depth=1.0, ctx: Context | None = None):
    """Mapping loss of Eq. 10 and Eq. 12 without the regulariser:
    w_color ((1 - lam) mean|C - C*| + lam (1 - SSIM(C, C*))) + w_depth mean|D - D*|.
    Returns (loss [1] device, dL/dcolor, dL/ddepth)."""
    loss, gC, gD = loss_l1(color, depth, tgt_color, tgt_depth, w_color * (1.0 - lam), w_depth, ctx=ctx)
    if lam != 0.0:
        loss_ssim(color, tgt_color, w_color * lam, loss, gC, ctx=ctx)
    return loss, gC, gD


def loss_track(color, depth, alpha, tgt_color, tgt_depth, lambda_c=0.5, inlier_mult=50.0, ctx: Context | None = None):
    """Tracking loss (Eq. 15); returns (loss [1], dL/dcolor, dL/ddepth, median [1])."""
    ctx = ctx or Context.get(color.device.index or 0)
    ctx.sync_stream()
    P_ = depth.numel()
    for t, nme in ((color, "color"), (depth, "depth"), (alpha, "alpha"), (tgt_color, "tgt_color"),
                   (tgt_depth, "tgt_depth")):
        _f32(t, nme)
    loss = torch.empty(1, device=color.device, dtype=torch.float32)
    med = torch.empty(1, device=color.device, dtype=torch.float32)
    gC = torch.empty_like(color)
    gD = torch.empty_like(depth)
    ctx.check(ctx.lib.gsr_loss_track(ctx.h, _ptr(color), _ptr(depth), _ptr(alpha), _ptr(tgt_color), _ptr(tgt_depth),
                                     P_, float(lambda_c), float(inlier_mult), _ptr(loss), _ptr(gC), _ptr(gD),
                                     _ptr(med)))
    return loss, gC, gD, med


def loss_track_noalloc(color, depth, alpha, tgt_color, tgt_depth, loss, dL_dcolor, dL_ddepth, median=None,
                       lambda_c=0.5, inlier_mult=50.0):
    """gsr_loss_track_noalloc: the tracking loss (Eq. 15) into caller-given
    outputs (loss [1], dL/dcolor, dL/ddepth, median [1] or None) on torch's
    current stream of the tensors' device; the library allocates nothing and
    needs no context (its scratch is a static device array shared by every
    call on the device)."""
    lib = load()
    P_ = depth.numel()
    for t, nme in ((color, "color"), (depth, "depth"), (alpha, "alpha"), (tgt_color, "tgt_color"),
                   (tgt_depth, "tgt_depth"), (loss, "loss"), (dL_dcolor, "dL_dcolor"), (dL_ddepth, "dL_ddepth")):
        _f32(t, nme)
    if median is not None:
        _f32(median, "median")
    if dL_dcolor.numel() != color.numel() or dL_ddepth.numel() != P_ or loss.numel() < 1:
        raise ValueError("output sizes do not match the inputs")
    with torch.cuda.device(color.device):
        stream = ctypes.c_void_p(torch.cuda.current_stream(color.device).cuda_stream)
        rc = lib.gsr_loss_track_noalloc(stream, _ptr(color), _ptr(depth), _ptr(alpha), _ptr(tgt_color),
                                        _ptr(tgt_depth), P_, float(lambda_c), float(inlier_mult), _ptr(loss),
                                        _ptr(dL_dcolor), _ptr(dL_ddepth), _ptr(median))
    if rc != 0:
        raise GsrError(rc, f"gsr_loss_track_noalloc: {lib.gsr_strerror(rc).decode()}: "
                           f"{lib.gsr_last_error(None).decode()}")


def adam_step(param, exp_avg, exp_avg_sq, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8,
              ctx: Context | None = None):
    ctx = ctx or Context.get(param.device.index or 0)
    ctx.sync_stream()
    for t, nme in ((param, "param"), (exp_avg, "exp_avg"), (exp_avg_sq, "exp_avg_sq"), (grad, "grad")):
        _f32(t, nme)
    ctx.check(ctx.lib.gsr_adam(ctx.h, _ptr(param), _ptr(exp_avg), _ptr(exp_avg_sq), _ptr(grad), param.numel(),
                               int(step), float(lr), float(beta1), float(beta2), float(eps)))


def profile_enable(on: bool = True, ctx: Context | None = None):
    ctx = ctx or Context.get(torch.cuda.current_device())
    ctx.check(ctx.lib.gsr_profile_enable(ctx.h, 1 if on else 0))


def profile_only(stage: str | None = None, ctx: Context | None = None):
    """Restricts stage timing to one stage (None: every stage)."""
    ctx = ctx or Context.get(torch.cuda.current_device())
    ctx.check(ctx.lib.gsr_profile_only(ctx.h, stage.encode() if stage else None))


def profile_read(ctx: Context | None = None) -> dict:
    """{stage: (total_ms, launches)} since the last read (synchronises)."""
    import numpy as np
    ctx = ctx or Context.get(torch.cuda.current_device())
    ctx.sync_stream()
    maxn = 64
    names = ctypes.create_string_buffer(32 * maxn)
    ms = np.zeros(maxn, np.float64)
    cnt = np.zeros(maxn, np.int64)
    n = ctypes.c_int()
    ctx.check(ctx.lib.gsr_profile_read(ctx.h, maxn, names, ms.ctypes.data_as(P), cnt.ctypes.data_as(P),
                                       ctypes.byref(n)))
    out = {}
    for i in range(min(n.value, maxn)):
        nm = names.raw[32 * i:32 * (i + 1)].split(b"\0")[0].decode()
        out[nm] = (float(ms[i]), int(cnt[i]))
    return out


def state_stats(state: State) -> dict:
    import numpy as np
    ctx = state.ctx
    ctx.sync_stream()
    out = np.zeros(6, np.int64)
    ctx.check(ctx.lib.gsr_state_stats(ctx.h, state.h, out.ctypes.data_as(P)))
    return dict(K=int(out[0]), visible=int(out[1]), pairs_fwd=int(out[2]), pairs_composited=int(out[3]),
                pairs_bwd=int(out[4]), tiles=int(out[5]))


def pose_const_velocity(pose_prev2, pose_prev1, ctx: Context | None = None):
    """Eq. 13 on the device: returns a new pose7 tensor."""
    ctx = ctx or Context.get(pose_prev1.device.index or 0)
    ctx.sync_stream()
    _f32(pose_prev2, "pose_prev2", (7,)); _f32(pose_prev1, "pose_prev1", (7,))
    out = torch.empty(7, device=pose_prev1.device, dtype=torch.float32)
    ctx.check(ctx.lib.gsr_pose_const_velocity(ctx.h, _ptr(pose_prev2), _ptr(pose_prev1), _ptr(out)))
    return out


class TrackGraph:
    """A captured tracking loop (n_iters iterations of render -> Eq. 15 loss ->
    pose backward -> Adam) over a frozen set of Gaussians."""

    def __init__(self, means, scales, quats, opacities, colors, camera: Camera, obs_color, obs_depth,
                 n_iters=100, lambda_c=0.5, inlier_mult=50.0, lr_q=5e-4, lr_t=1e-3, betas=(0.9, 0.999), eps=1e-8,
                 K_cap: int = 0, opts: RasterOpts | None = None, ctx: Context | None = None):
        self.ctx = ctx or Context.get(means.device.index or 0)
        self.ctx.sync_stream()
        self.keep = (means, scales, quats, opacities, colors)
        g = _gaussians(means, scales, quats, opacities, colors)
        self.n_iters = int(n_iters)
        to = TrackOpts(lambda_c, inlier_mult, lr_q, lr_t, betas[0], betas[1], eps, self.n_iters)
        oc = (opts or RasterOpts()).c()
        self.h = P()
        _f32(obs_color, "obs_color"); _f32(obs_depth, "obs_depth")
        self.ctx.check(self.ctx.lib.gsr_track_graph_create(self.ctx.h, ctypes.byref(g), ctypes.byref(camera),
                                                           ctypes.byref(oc), ctypes.byref(to), _ptr(obs_color),
                                                           _ptr(obs_depth), int(K_cap), ctypes.byref(self.h)))

    def set_frame(self, obs_color, obs_depth):
        self.ctx.sync_stream()
        _f32(obs_color, "obs_color"); _f32(obs_depth, "obs_depth")
        self.ctx.check(self.ctx.lib.gsr_track_graph_set_frame(self.ctx.h, self.h, _ptr(obs_color), _ptr(obs_depth)))

    def run(self, pose7, losses=None):
        """Optimise pose7 (device, in place); optionally fill losses [n_iters]."""
        self.ctx.sync_stream()
        _f32(pose7, "pose7", (7,))
        if losses is not None:
            _f32(losses, "losses", (self.n_iters,))
        self.ctx.check(self.ctx.lib.gsr_track_graph_run(self.ctx.h, self.h, _ptr(pose7), _ptr(losses)))
        return pose7

    def close(self):
        if self.h is not None and self.h.value:
            self.ctx.lib.gsr_track_graph_destroy(self.ctx.h, self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pose_adam_step(pose7, state, grad7, lr_q, lr_t, beta1=0.9, beta2=0.999, eps=1e-8, ctx: Context | None = None):
    """In-place Adam step on a pose7; state: zero-initialised float32 [20] device tensor."""
    ctx = ctx or Context.get(pose7.device.index or 0)
    ctx.sync_stream()
    _f32(pose7, "pose7", (7,)); _f32(state, "state", (20,)); _f32(grad7, "grad7", (7,))
    ctx.check(ctx.lib.gsr_pose_adam(ctx.h, _ptr(pose7), _ptr(state), _ptr(grad7), float(lr_q), float(lr_t),
                                    float(beta1), float(beta2), float(eps)))


class InitNet:
    """Handle of the tracking-initialisation CNN (BF16 MFMA kernels in libgsr)."""

    IN_H, IN_W, IN_C = 120, 160, 8

    def __init__(self, max_batch: int, ctx: Context | None = None):
        self.ctx = ctx or Context.get(torch.cuda.current_device())
        self.ctx.sync_stream()
        self.max_batch = int(max_batch)
        self.h = P()
        self.ctx.check(self.ctx.lib.gsr_initnet_create(self.ctx.h, self.max_batch, ctypes.byref(self.h)))
        n = ctypes.c_int64()
        self.ctx.check(self.ctx.lib.gsr_initnet_count(self.ctx.h, self.h, ctypes.byref(n)))
        self.n_params = int(n.value)

    def set_params(self, flat):
        self.ctx.sync_stream()
        _f32(flat, "params", (self.n_params,))
        self.ctx.check(self.ctx.lib.gsr_initnet_set_params(self.ctx.h, self.h, _ptr(flat)))

    def get_params(self, with_grads=False):
        self.ctx.sync_stream()
        p = torch.empty(self.n_params, device="cuda", dtype=torch.float32)
        g = torch.empty(self.n_params, device="cuda", dtype=torch.float32) if with_grads else None
        self.ctx.check(self.ctx.lib.gsr_initnet_get_params(self.ctx.h, self.h, _ptr(p), _ptr(g)))
        return (p, g) if with_grads else p

    def set_input(self, x):
        """x: BF16 [B,120,160,8] device tensor."""
        self.ctx.sync_stream()
        if x.dtype != torch.bfloat16 or not x.is_contiguous() or tuple(x.shape[1:]) != (self.IN_H, self.IN_W, self.IN_C):
            raise ValueError("input must be a contiguous bfloat16 [B,120,160,8] tensor")
        self.ctx.check(self.ctx.lib.gsr_initnet_set_input(self.ctx.h, self.h, x.shape[0], _ptr(x)))

    def activation(self, layer: int, batch: int, shape):
        self.ctx.sync_stream()
        a = torch.empty((batch,) + tuple(shape), device="cuda", dtype=torch.bfloat16)
        d = torch.empty_like(a)
        self.ctx.check(self.ctx.lib.gsr_initnet_get_activation(self.ctx.h, self.h, layer, batch, _ptr(a), _ptr(d)))
        return a, d

    def forward(self, batch: int):
        self.ctx.sync_stream()
        out = torch.empty((batch, 6), device="cuda", dtype=torch.float32)
        self.ctx.check(self.ctx.lib.gsr_initnet_forward(self.ctx.h, self.h, batch, _ptr(out)))
        return out

    def backward(self, batch: int, labels=None, scale=None, dL_dout=None):
        self.ctx.sync_stream()
        loss = torch.zeros(1, device="cuda", dtype=torch.float32)
        self.ctx.check(self.ctx.lib.gsr_initnet_backward(self.ctx.h, self.h, batch, _ptr(labels), _ptr(scale),
                                                         _ptr(dL_dout), _ptr(loss)))
        return loss

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.ctx.sync_stream()
        self.ctx.check(self.ctx.lib.gsr_initnet_adam(self.ctx.h, self.h, float(lr), float(beta1), float(beta2),
                                                     float(eps)))

    def close(self):
        if self.h is not None and self.h.value:
            self.ctx.lib.gsr_initnet_destroy(self.ctx.h, self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_rgbd_pair(rend_color, rend_depth, obs_color, obs_depth, dst, depth_scale=0.25, ctx: Context | None = None):
    """Pack one sample into dst (BF16 [120,160,8] device tensor view)."""
    ctx = ctx or Context.get(rend_color.device.index or 0)
    ctx.sync_stream()
    H, W = rend_depth.shape
    if dst.dtype != torch.bfloat16 or not dst.is_contiguous():
        raise ValueError("dst must be a contiguous bfloat16 tensor")
    ctx.check(ctx.lib.gsr_pack_rgbd_pair(ctx.h, _ptr(rend_color), _ptr(rend_depth), _ptr(obs_color), _ptr(obs_depth),
                                         H, W, float(depth_scale), _ptr(dst)))


def pose_apply_twist(pose7, twist6, ctx: Context | None = None):
    """exp(twist^) T on the device; returns a new pose7 tensor."""
    ctx = ctx or Context.get(pose7.device.index or 0)
    ctx.sync_stream()
    _f32(pose7, "pose7", (7,)); _f32(twist6, "twist6", (6,))
    out = torch.empty(7, device=pose7.device, dtype=torch.float32)
    ctx.check(ctx.lib.gsr_pose_apply_twist(ctx.h, _ptr(pose7), _ptr(twist6), _ptr(out)))
    return out


def adam_groups(params, exp_avgs, exp_avg_sqs, grads, lrs, step, beta1=0.9, beta2=0.999, eps=1e-8,
                ctx: Context | None = None):
    """One fused Adam launch over several float32 device tensors (<= 8)."""
    ctx = ctx or Context.get(params[0].device.index or 0)
    ctx.sync_stream()
    n = len(params)
    arr = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])
    for group in (params, exp_avgs, exp_avg_sqs, grads):
        for t in group:
            _f32(t, "adam tensor")
    counts = (ctypes.c_int64 * n)(*[t.numel() for t in params])
    lr = (ctypes.c_float * n)(*[float(x) for x in lrs])
    ctx.check(ctx.lib.gsr_adam_groups(ctx.h, n, arr(params), arr(exp_avgs), arr(exp_avg_sqs), arr(grads),
                                      ctypes.cast(counts, P), ctypes.cast(lr, P), int(step), float(beta1),
                                      float(beta2), float(eps)))
