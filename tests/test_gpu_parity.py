"""HIP path vs the FP64 oracle, through the C ABI (config C1 and edge cases).

Bars: tile lists bit-exact (inputs certified by the oracle), colour / depth /
alpha within 1e-4 absolute, gradients within 1e-3 relative plus a floor of
1e-5 of the sum of absolute per-pixel terms (and the ambiguity slack)."""
import numpy as np
import pytest

import oracle
from paper_2312_10070_amd import gsr, synth
from tests import gpu_cases as G
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = {"color": 1e-4, "depth": 1e-4, "alpha": 1e-4}
C1_OPTS = oracle.Opts(amb_z=0.0)  # identity pose: the FP32 camera depth equals the input depth exactly
SHAPES = [(16, 16), (8, 32), (32, 8)]


def torch_():
    import torch
    return torch


def run_fwd(g, pose, cam: oracle.Camera, tw=16, th=16):
    torch = torch_()
    d = G.to_dev(g)
    pose_d = torch.tensor(np.asarray(pose, np.float32), device="cuda")
    camera = gsr.make_camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.near_z, cam.bg)
    opts = gsr.RasterOpts(tile_w=tw, tile_h=th)
    color, depth, alpha, st = gsr.render_fwd(d["means"], d["scales"], d["quats"], d["opacities"], d["colors"],
                                             pose_d, camera, opts)
    torch.cuda.synchronize()
    return dict(color=color.cpu().numpy(), depth=depth.cpu().numpy(), alpha=alpha.cpu().numpy()), st, d, pose_d


def test_c1_tile_lists_bit_exact():
    g, _, pose, cam = G.c1_case(0)
    for tw, th in SHAPES:
        out, st, _, _ = run_fwd(g, pose, cam, tw, th)
        tl = oracle.tile_lists(g, pose, cam, oracle.Opts(tile_w=tw, tile_h=th))
        K, ranges, ids = gsr.tile_lists(st, tl["ranges"].shape[0])
        assert K == tl["K"]
        G.compare_tile_lists(ranges.cpu().numpy(), ids.cpu().numpy(), tl, None, strict=True)


def test_c1_forward_parity_all_tile_shapes_bitwise_equal():
    g, _, pose, cam = G.c1_case(0)
    orc = oracle.render(g, pose, cam, C1_OPTS)
    imgs = []
    for tw, th in SHAPES:
        out, _, _, _ = run_fwd(g, pose, cam, tw, th)
        G.compare_images(out, orc, TOL)
        imgs.append(out)
    for other in imgs[1:]:
        for k in ("color", "depth", "alpha"):
            assert np.array_equal(imgs[0][k], other[k]), f"{k} depends on the tile shape"


def test_c1_permutation_invariance_bitwise():
    g, _, pose, cam = G.c1_case(1)
    perm = np.random.default_rng(0).permutation(len(g["means"]))
    a, _, _, _ = run_fwd(g, pose, cam)
    b, _, _, _ = run_fwd({k: v[perm] for k, v in g.items()}, pose, cam)
    for k in ("color", "depth", "alpha"):
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c1_backward_parity(seed):
    torch = torch_()
    g, tg, pose, cam = G.c1_case(seed)
    opts = C1_OPTS
    orc = oracle.render(g, pose, cam, opts)
    tgt = oracle.render(tg, pose, cam, opts)
    # upstream gradients: the oracle's mapping L1 loss, cast to FP32 for both sides
    _, gC, gD = oracle.loss_l1(orc["color"].astype(np.float32), orc["depth"].astype(np.float32),
                               tgt["color"].astype(np.float32), tgt["depth"].astype(np.float32))
    gC32, gD32 = gC.astype(np.float32), gD.astype(np.float32)
    rng = np.random.default_rng(seed)
    gA32 = (rng.normal(size=gD.shape) * 1e-4).astype(np.float32)
    ref = oracle.backward(g, pose, cam, opts, gC32.astype(np.float64), gD32.astype(np.float64),
                          gA32.astype(np.float64))
    _, st, _, _ = run_fwd(g, pose, cam)
    out = gsr.render_bwd(st, torch.from_numpy(gC32).cuda(), torch.from_numpy(gD32).cuda(),
                         torch.from_numpy(gA32).cuda())
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    case = f"C1 seed {seed}"
    G.grads_check(got, ref, case=case)
    H.check_grad_ref("pose7", got["pose7"], ref, case=case)
    H.check_grad_ref("twist6", got["twist6"], ref, case=case)


def posed_case(seed=3, n=2000, W=70, Hh=50):
    """Non-identity pose, non-zero background, ragged tiles (70 x 50)."""
    rng = np.random.default_rng(seed)
    g = dict(means=np.stack([rng.uniform(-1.2, 1.2, n), rng.uniform(-0.9, 0.9, n), rng.uniform(1, 5, n)], 1),
             scales=np.exp(rng.normal(-3.0, 0.4, (n, 3))), quats=rng.normal(size=(n, 4)),
             opacities=1 / (1 + np.exp(-rng.normal(0, 1, n))), colors=rng.uniform(0, 1, (n, 3)))
    g["scales"][:5] = 0.6  # a few large Gaussians spanning many tiles
    cam = oracle.Camera(W, Hh, 55.0, 57.0, 34.3, 26.1, 0.2, (0.2, 0.5, 0.1))
    pose = np.array([0.995, 0.04, -0.06, 0.03, 0.05, -0.04, 0.2])
    pose[:4] /= np.linalg.norm(pose[:4])
    pose = pose.astype(np.float32).astype(np.float64)
    g = G.certify(g, pose, cam, 2e-4)
    return g, pose, cam


def test_posed_ragged_forward_backward_and_tiles():
    torch = torch_()
    g, pose, cam = posed_case()
    opts = oracle.Opts(amb_rel=1e-4)
    orc = oracle.render(g, pose, cam, opts)
    for tw, th in SHAPES:
        out, st, _, _ = run_fwd(g, pose, cam, tw, th)
        G.compare_images(out, orc, TOL)
        tl = oracle.tile_lists(g, pose, cam, oracle.Opts(tile_w=tw, tile_h=th))
        K, ranges, ids = gsr.tile_lists(st, tl["ranges"].shape[0])
        rec = oracle.project(g, pose, cam, oracle.Opts())
        G.compare_tile_lists(ranges.cpu().numpy(), ids.cpu().numpy(), tl, rec["z_cam"], strict=False)
    rng = np.random.default_rng(1)
    gC = (rng.normal(size=(3, cam.height, cam.width)) * 1e-3).astype(np.float32)
    gD = (rng.normal(size=(cam.height, cam.width)) * 1e-3).astype(np.float32)
    ref = oracle.backward(g, pose, cam, opts, gC.astype(np.float64), gD.astype(np.float64))
    _, st, _, _ = run_fwd(g, pose, cam)
    out = gsr.render_bwd(st, torch.from_numpy(gC).cuda(), torch.from_numpy(gD).cuda())
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    case = "posed 70x50"
    G.grads_check(got, ref, case=case)
    H.check_grad_ref("pose7", got["pose7"], ref, case=case)
    H.check_grad_ref("twist6", got["twist6"], ref, case=case)
    # pose only: the six-field reduction (no opacity / colour fields)
    out_p = gsr.render_bwd(st, torch.from_numpy(gC).cuda(), torch.from_numpy(gD).cuda(), want_params=False)
    torch.cuda.synchronize()
    for k in ("pose7", "twist6"):
        gp = out_p[k].cpu().numpy().astype(np.float64)
        H.check_grad_ref(k, gp, ref, case=case + " six-field")


def test_frame_with_more_tiles_than_one_binning_chunk():
    """2100 x 2100 = 132 x 132 = 17424 tiles, more than one counting / placing
    workgroup's LDS tile chunk (16384): binning runs with two tile chunks per
    workgroup column. Tile lists against the oracle, sampled pixels of the
    forward and a second forward on the same state (the range scan's tile
    totals and ticket must have returned to zero)."""
    rng = np.random.default_rng(8)
    n = 4000
    g = dict(means=np.stack([rng.uniform(-1.3, 1.3, n), rng.uniform(-1.3, 1.3, n), rng.uniform(1.5, 4, n)], 1),
             scales=np.exp(rng.normal(-3.5, 0.5, (n, 3))), quats=rng.normal(size=(n, 4)),
             opacities=1 / (1 + np.exp(-rng.normal(0, 1, n))), colors=rng.uniform(0, 1, (n, 3)))
    g["scales"][:3] = 0.8  # a few Gaussians spanning both chunks
    cam = oracle.Camera(2100, 2100, 1500.0, 1500.0, 1050.3, 1049.7, 0.2, (0.1, 0.2, 0.3))
    pose = np.array([0.999, 0.02, -0.03, 0.01, 0.02, -0.01, 0.1])
    pose[:4] /= np.linalg.norm(pose[:4])
    pose = pose.astype(np.float32).astype(np.float64)
    g = G.certify(g, pose, cam, 2e-4)
    tl = oracle.tile_lists(g, pose, cam, oracle.Opts())
    assert tl["ranges"].shape[0] == 17424
    rec = oracle.project(g, pose, cam, oracle.Opts())
    pixels = np.sort(rng.choice(cam.width * cam.height, 3000, replace=False))
    orc = oracle.render(g, pose, cam, oracle.Opts(amb_rel=1e-4), pixels=pixels, nthreads=8)
    yy, xx = pixels // cam.width, pixels % cam.width
    sub_o = {k: (v[:, yy, xx] if v.ndim == 3 else v[yy, xx]) for k, v in orc.items() if k != "hash"}
    for rep in range(2):
        out, st, _, _ = run_fwd(g, pose, cam)
        K, ranges, ids = gsr.tile_lists(st, tl["ranges"].shape[0])
        assert K == tl["K"]
        G.compare_tile_lists(ranges.cpu().numpy(), ids.cpu().numpy(), tl, rec["z_cam"], strict=False)
        sub_g = {k: (v[:, yy, xx] if v.ndim == 3 else v[yy, xx]) for k, v in out.items()}
        G.compare_images(sub_g, sub_o, TOL)
        st.release()


def test_empty_and_fully_culled_inputs_render_background():
    cam = oracle.Camera(40, 30, 30.0, 30.0, 20.0, 15.0, 0.2, (0.3, 0.6, 0.9))
    pose = np.array([1, 0, 0, 0, 0, 0, 0], np.float64)
    empty = {k: np.zeros(s, np.float32) for k, s in (("means", (0, 3)), ("scales", (0, 3)), ("quats", (0, 4)),
                                                     ("opacities", (0,)), ("colors", (0, 3)))}
    torch = torch_()
    out, st, _, _ = run_fwd(empty, pose, cam)
    for ch, v in enumerate((0.3, 0.6, 0.9)):
        assert np.all(out["color"][ch] == np.float32(v))
    assert not out["depth"].any() and not out["alpha"].any()
    b = gsr.render_bwd(st, torch.ones((3, 30, 40), device="cuda"), torch.ones((30, 40), device="cuda"))
    torch.cuda.synchronize()
    assert not b["pose7"].cpu().numpy().any()
    n = 50
    behind = dict(means=np.tile([0, 0, -1.0], (n, 1)), scales=np.full((n, 3), 0.1), quats=np.tile([1.0, 0, 0, 0], (n, 1)),
                  opacities=np.full(n, 0.9), colors=np.ones((n, 3)))
    out, st, _, _ = run_fwd(G.f32(behind), pose, cam)
    assert not out["alpha"].any()
    K, _, _ = gsr.tile_lists(st, 6)
    assert K == 0
    zero_o = dict(behind)
    zero_o["means"] = np.tile([0, 0, 2.0], (n, 1))
    zero_o["opacities"] = np.zeros(n)
    out, _, _, _ = run_fwd(G.f32(zero_o), pose, cam)
    assert not out["alpha"].any()


def test_long_lists_and_early_termination():
    """Hundreds of large opaque Gaussians on every tile: lists span several LDS
    batches and every pixel terminates early."""
    rng = np.random.default_rng(7)
    n = 3000
    g = dict(means=np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.4, 0.4, n), rng.uniform(2, 3, n)], 1),
             scales=np.exp(rng.normal(-1.5, 0.2, (n, 3))), quats=rng.normal(size=(n, 4)),
             opacities=rng.uniform(0.3, 0.9, n), colors=rng.uniform(0, 1, (n, 3)))
    cam = oracle.Camera(48, 40, 40.0, 40.0, 24.0, 20.0)
    pose = np.array([1, 0, 0, 0, 0, 0, 0], np.float64)
    g = G.certify(g, pose, cam, 1e-4)
    opts = oracle.Opts(amb_rel=1e-4, amb_z=0.0)  # identity pose: FP32 depth is exact
    orc = oracle.render(g, pose, cam, opts)
    out, st, _, _ = run_fwd(g, pose, cam)
    G.compare_images(out, orc, TOL)
    tl = oracle.tile_lists(g, pose, cam, oracle.Opts())
    assert (tl["ranges"][:, 1] - tl["ranges"][:, 0]).max() > 600
    assert (orc["alpha"] > 1 - 2e-4).mean() > 0.3
    torch = torch_()
    rng = np.random.default_rng(2)
    gC = (rng.normal(size=(3, 40, 48)) * 1e-3).astype(np.float32)
    gD = (rng.normal(size=(40, 48)) * 1e-3).astype(np.float32)
    ref = oracle.backward(g, pose, cam, opts, gC.astype(np.float64), gD.astype(np.float64))
    b = gsr.render_bwd(st, torch.from_numpy(gC).cuda(), torch.from_numpy(gD).cuda())
    torch.cuda.synchronize()
    G.grads_check({k: v.cpu().numpy().astype(np.float64) for k, v in b.items()}, ref, case="long lists 48x40")


def test_tile_ranges_longer_than_one_wave_are_merged():
    """Tiles whose lists exceed the 2048 keys one wave sorts in registers
    (runs of 1024 keys sorted by the workgroup's waves side by side, more runs
    than waves in one workgroup, merged pairwise in global memory, with a
    ragged last run): tile lists bit-exact, including depth ties broken by
    index."""
    rng = np.random.default_rng(11)
    n = 7000
    g = dict(means=np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.25, 0.25, n), rng.uniform(2, 6, n)], 1),
             scales=np.exp(rng.normal(-2.2, 0.3, (n, 3))), quats=rng.normal(size=(n, 4)),
             opacities=rng.uniform(0.2, 0.9, n), colors=rng.uniform(0, 1, (n, 3)))
    g["means"][100:400, 2] = 3.0  # exact depth ties: order by index
    cam = oracle.Camera(48, 40, 40.0, 40.0, 24.0, 20.0)
    pose = np.array([1, 0, 0, 0, 0, 0, 0], np.float64)
    g = G.certify(g, pose, cam, 1e-4)
    tl = oracle.tile_lists(g, pose, cam, oracle.Opts())
    lens = tl["ranges"][:, 1] - tl["ranges"][:, 0]
    assert lens.max() > 2 * 2048 + 100 and (lens > 2048).sum() >= 2
    runs = np.where(lens > 2048, (lens + 1023) // 1024, 0)
    assert max(runs[i:i + 4].sum() for i in range(0, len(runs), 4)) > 4  # four tiles (waves) per workgroup
    out, st, _, _ = run_fwd(g, pose, cam)
    K, ranges, ids = gsr.tile_lists(st, tl["ranges"].shape[0])
    assert K == tl["K"]
    G.compare_tile_lists(ranges.cpu().numpy(), ids.cpu().numpy(), tl, None)
    # 7000 Gaussians over 1920 pixels: many threshold events, so a looser unverifiable bound
    opts = oracle.Opts(amb_rel=1e-4, amb_z=0.0)
    G.compare_images(out, oracle.render(g, pose, cam, opts), TOL, max_unverifiable=0.06)


def test_register_sorts_of_long_tile_lists():
    """Tile lists of 513..1024 and 1025..2048 keys, sorted by one wave in
    registers (16 and 32 keys per lane): bit-exact, including depth ties."""
    rng = np.random.default_rng(12)
    n = 1500
    g = dict(means=np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.25, 0.25, n), rng.uniform(2, 6, n)], 1),
             scales=np.exp(rng.normal(-2.2, 0.3, (n, 3))), quats=rng.normal(size=(n, 4)),
             opacities=rng.uniform(0.2, 0.9, n), colors=rng.uniform(0, 1, (n, 3)))
    g["means"][50:150, 2] = 3.0  # exact depth ties: order by index
    cam = oracle.Camera(48, 40, 40.0, 40.0, 24.0, 20.0)
    pose = np.array([1, 0, 0, 0, 0, 0, 0], np.float64)
    g = G.certify(g, pose, cam, 1e-4)
    tl = oracle.tile_lists(g, pose, cam, oracle.Opts())
    lens = tl["ranges"][:, 1] - tl["ranges"][:, 0]
    assert ((lens > 512) & (lens <= 1024)).any() and ((lens > 1024) & (lens <= 2048)).any(), lens
    _, st, _, _ = run_fwd(g, pose, cam)
    K, ranges, ids = gsr.tile_lists(st, tl["ranges"].shape[0])
    assert K == tl["K"]
    G.compare_tile_lists(ranges.cpu().numpy(), ids.cpu().numpy(), tl, None)


def tile_stacks(lengths, seed=0, tie_every=7):
    """Gaussians stacked on the centres of the tiles of a 48x48 frame (3 x 3
    tiles of 16 x 16): lengths[t] small Gaussians (projected radius well under a
    pixel, centres within 2 px of the tile centre) at random depths in [2, 6],
    every tie_every-th one sharing the depth of the one before (ties broken by
    index), so tile t's list has exactly lengths[t] keys."""
    rng = np.random.default_rng(seed)
    cam = oracle.Camera(48, 48, 40.0, 40.0, 24.0, 24.0)
    means = []
    for t, L in enumerate(lengths):
        u = 16 * (t % 3) + 7.5 + rng.uniform(-2, 2, L)
        v = 16 * (t // 3) + 7.5 + rng.uniform(-2, 2, L)
        z = rng.uniform(2, 6, L)
        z[tie_every::tie_every] = z[tie_every - 1:-1:tie_every][:len(z[tie_every::tie_every])]
        means.append(np.stack([(u - cam.cx) / cam.fx * z, (v - cam.cy) / cam.fy * z, z], 1))
    means = np.concatenate(means)
    n = len(means)
    g = dict(means=means, scales=np.full((n, 3), 0.004), quats=rng.normal(size=(n, 4)),
             opacities=rng.uniform(0.3, 0.9, n), colors=rng.uniform(0, 1, (n, 3)))
    return g, cam


def test_tile_sort_length_boundaries():
    """Tiles of exactly 0, 1, 512, 513, 1024, 1025, 2048, 2049 and 4097 keys:
    the edges of the 512 / 1024 / 2048-key register networks and of the runs of
    1024 keys (a run of one key; five runs in a workgroup of four waves), in
    one frame; tile lists bit-exact against the oracle, including depth ties."""
    lengths = [2048, 2049, 1025, 1024, 513, 512, 4097, 1, 0]
    g, cam = tile_stacks(lengths)
    pose = np.array([1, 0, 0, 0, 0, 0, 0], np.float64)
    g = G.certify(g, pose, cam, 1e-4)
    tl = oracle.tile_lists(g, pose, cam, oracle.Opts())
    lens = tl["ranges"][:, 1] - tl["ranges"][:, 0]
    assert lens.tolist() == lengths, lens
    _, st, _, _ = run_fwd(g, pose, cam)
    K, ranges, ids = gsr.tile_lists(st, tl["ranges"].shape[0])
    assert K == tl["K"] == sum(lengths)
    G.compare_tile_lists(ranges.cpu().numpy(), ids.cpu().numpy(), tl, None)


def test_workspace_growth_between_calls():
    """A forward whose overlap count exceeds the tile-list workspace left by the
    previous forward on the same (reused) state: the speculatively queued
    second half is redone with a larger workspace, and the lists and image
    still match the oracle."""
    g, _, pose, cam = G.c1_case(0, n=200)
    out, st, _, _ = run_fwd(g, pose, cam)
    k_small = gsr.tile_lists(st, 12)[0]
    st.release()
    g2, _, _, _ = G.c1_case(1, n=3000)
    g2["scales"] = (g2["scales"] * 3.0).astype(np.float32)
    g2 = G.certify(g2, pose, cam, 1e-4)
    out2, st2, _, _ = run_fwd(g2, pose, cam)
    tl = oracle.tile_lists(g2, pose, cam, oracle.Opts())
    assert tl["K"] > 2 * k_small
    K, ranges, ids = gsr.tile_lists(st2, tl["ranges"].shape[0])
    assert K == tl["K"]
    G.compare_tile_lists(ranges.cpu().numpy(), ids.cpu().numpy(), tl, None)
    G.compare_images(out2, oracle.render(g2, pose, cam, C1_OPTS), TOL, max_unverifiable=0.02)


def test_loss_kernels_match_oracle():
    torch = torch_()
    g, tg, pose, cam = G.c1_case(0)
    out, _, _, _ = run_fwd(g, pose, cam)
    tgt = oracle.render(tg, pose, cam, oracle.Opts())
    Ct = tgt["color"].astype(np.float32)
    Dt = tgt["depth"].astype(np.float32)
    Dt[:4] = 0.0  # invalid observed depth rows for the tracking mask
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    loss, gC, gD = gsr.loss_l1(dev(out["color"]), dev(out["depth"]), dev(Ct), dev(Dt), 0.8, 1.2)
    L_ref, gC_ref, gD_ref = oracle.loss_l1(out["color"], out["depth"], Ct, Dt, 0.8, 1.2)
    torch.cuda.synchronize()
    assert abs(loss.item() - L_ref) <= 1e-5 * abs(L_ref)
    np.testing.assert_allclose(gC.cpu().numpy(), gC_ref, rtol=1e-6, atol=0)
    np.testing.assert_allclose(gD.cpu().numpy(), gD_ref, rtol=1e-6, atol=0)
    loss, gC, gD, med = gsr.loss_track(dev(out["color"]), dev(out["depth"]), dev(out["alpha"]), dev(Ct), dev(Dt),
                                       0.5, 50.0)
    r = oracle.loss_track(out["color"], out["depth"], out["alpha"], Ct, Dt, 0.5, 50.0)
    torch.cuda.synchronize()
    assert med.item() == r["median"]  # the median is an exact element
    assert abs(loss.item() - r["loss"]) <= 1e-5 * abs(r["loss"]) + 1e-9
    np.testing.assert_allclose(gC.cpu().numpy(), r["gC"], rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(gD.cpu().numpy(), r["gD"], rtol=1e-5, atol=1e-9)


def track_images(rng, h, w, invalid=0.0):
    C = rng.uniform(0, 1, (3, h, w)).astype(np.float32)
    Ct = rng.uniform(0, 1, (3, h, w)).astype(np.float32)
    D = rng.uniform(1, 3, (h, w)).astype(np.float32)
    Dt = (D + rng.normal(0, 0.05, (h, w))).astype(np.float32)
    A = rng.uniform(0.3, 1.0, (h, w)).astype(np.float32)
    Dt[rng.uniform(size=(h, w)) < invalid] = 0.0
    return C, D, A, Ct, Dt


@pytest.mark.parametrize("case", ["one_pixel", "no_valid_pixel", "two_valid_lower_middle", "all_equal",
                                  "all_zero_error", "six_decades", "ragged_37x23"])
def test_loss_track_edge_cases(case):
    """Eq. 15 (with the supplement's masks) on the degenerate inputs of its
    exact median: a single pixel, no valid observed depth, an even count (the
    lower middle), every error equal or zero, errors spread over six decades,
    a ragged frame with invalid pixels. The median is compared bit for bit,
    the loss and gradients per element."""
    torch = torch_()
    rng = np.random.default_rng(sum(map(ord, case)))
    if case == "one_pixel":
        C, D, A, Ct, Dt = track_images(rng, 1, 1)
    elif case == "no_valid_pixel":
        C, D, A, Ct, Dt = track_images(rng, 4, 6)
        Dt[:] = 0.0
    elif case == "two_valid_lower_middle":
        C, D, A, Ct, Dt = track_images(rng, 3, 5)
        Dt[:] = 0.0
        Dt[0, 1], Dt[2, 3] = D[0, 1] + 0.25, D[2, 3] - 0.5
    elif case == "all_equal":
        C, D, A, Ct, Dt = track_images(rng, 5, 7)
        Dt[:] = D + np.float32(0.125)
    elif case == "all_zero_error":
        C, D, A, Ct, Dt = track_images(rng, 6, 6)
        Dt[:] = D
    elif case == "six_decades":
        C, D, A, Ct, Dt = track_images(rng, 16, 16)
        D[:] = np.float32(1e3)
        Dt[:] = (D - np.exp(rng.uniform(np.log(1e-3), np.log(999.0), D.shape))).astype(np.float32)
    else:
        C, D, A, Ct, Dt = track_images(rng, 23, 37, invalid=0.1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    loss, gC, gD, med = gsr.loss_track(dev(C), dev(D), dev(A), dev(Ct), dev(Dt), 0.5, 50.0)
    torch.cuda.synchronize()
    r = oracle.loss_track(C, D, A, Ct, Dt, 0.5, 50.0)
    if case == "no_valid_pixel":
        assert r["n_inlier"] == 0 and r["loss"] == 0.0
    assert med.item() == r["median"]
    assert abs(loss.item() - r["loss"]) <= 1e-5 * abs(r["loss"]) + 1e-9
    np.testing.assert_allclose(gC.cpu().numpy(), r["gC"], rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(gD.cpu().numpy(), r["gD"], rtol=1e-5, atol=1e-9)


def test_adam_matches_oracle():
    torch = torch_()
    rng = np.random.default_rng(0)
    p = rng.normal(size=64)
    m = np.zeros(64); v = np.zeros(64)
    pd = torch.tensor(p, dtype=torch.float32, device="cuda")
    md = torch.zeros(64, device="cuda"); vd = torch.zeros(64, device="cuda")
    for step in range(1, 31):
        gr = rng.normal(size=64).astype(np.float32)
        oracle.adam(p, m, v, gr.astype(np.float64), step, 1e-2)
        gsr.adam_step(pd, md, vd, torch.from_numpy(gr).cuda(), step, 1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pd.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


def test_invalid_arguments_are_rejected():
    torch = torch_()
    cam = gsr.make_camera(32, 32, 30, 30, 16, 16)
    d = G.to_dev(dict(means=np.zeros((1, 3)), scales=np.ones((1, 3)), quats=np.array([[1.0, 0, 0, 0]]),
                      opacities=np.ones(1) * 0.5, colors=np.ones((1, 3))))
    pose = torch.tensor([1, 0, 0, 0, 0, 0, 0], dtype=torch.float32, device="cuda")
    with pytest.raises(gsr.GsrError) as e:
        gsr.render_fwd(d["means"], d["scales"], d["quats"], d["opacities"], d["colors"], pose, cam,
                       gsr.RasterOpts(tile_w=16, tile_h=8))
    assert e.value.code == gsr.GSR_EINVAL
    bad = gsr.make_camera(0, 32, 30, 30, 16, 16)
    with pytest.raises(gsr.GsrError):
        gsr.render_fwd(d["means"], d["scales"], d["quats"], d["opacities"], d["colors"], pose, bad)
    nan_cam = gsr.make_camera(32, 32, float("nan"), 30, 16, 16)
    with pytest.raises(gsr.GsrError):
        gsr.render_fwd(d["means"], d["scales"], d["quats"], d["opacities"], d["colors"], pose, nan_cam)


def test_fused_adam_groups_match_oracle():
    torch = torch_()
    rng = np.random.default_rng(5)
    sizes = [7, 300, 1, 64]
    lrs = [1e-2, 3e-3, 5e-2, 1e-4]
    ps = [rng.normal(size=n) for n in sizes]
    ms = [np.zeros(n) for n in sizes]; vs = [np.zeros(n) for n in sizes]
    pd = [torch.tensor(p, dtype=torch.float32, device="cuda") for p in ps]
    md = [torch.zeros(n, device="cuda") for n in sizes]; vd = [torch.zeros(n, device="cuda") for n in sizes]
    for step in range(1, 11):
        gs = [rng.normal(size=n).astype(np.float32) for n in sizes]
        for p, m, v, g, lr in zip(ps, ms, vs, gs, lrs):
            oracle.adam(p, m, v, g.astype(np.float64), step, lr)
        gsr.adam_groups(pd, md, vd, [torch.from_numpy(g).cuda() for g in gs], lrs, step)
    torch.cuda.synchronize()
    for p, d in zip(ps, pd):
        np.testing.assert_allclose(d.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


def test_stage_profile_filter():
    """gsr_profile_only: with a filter only that stage is timed; without, every
    stage of the call is."""
    g, _, pose, cam = G.c1_case(0)
    gsr.profile_read()
    try:
        gsr.profile_only("render_fwd")
        gsr.profile_enable(True)
        _, st, _, _ = run_fwd(g, pose, cam)
        st.release()
        gsr.profile_enable(False)
        only = gsr.profile_read()
        assert set(only) == {"render_fwd"} and only["render_fwd"][1] == 1 and only["render_fwd"][0] > 0
        gsr.profile_only(None)
        gsr.profile_enable(True)
        _, st, _, _ = run_fwd(g, pose, cam)
        st.release()
        gsr.profile_enable(False)
        every = gsr.profile_read()
        assert {"project", "bin_count", "tile_bins", "render_fwd"} <= set(every)
        with pytest.raises(gsr.GsrError):
            gsr.profile_only("x" * 40)
    finally:
        gsr.profile_enable(False)
        gsr.profile_only(None)
        gsr.profile_read()


def test_backward_fused_with_adam_matches_separate_calls():
    """gsr_render_bwd_adam equals gsr_render_bwd followed by gsr_adam_groups
    (single view and a two-view batch); up to the order of the compositing
    backward's float atomics, which reaches the update only through rounding."""
    torch = torch_()
    g, tg, pose, cam = G.c1_case(0)
    camera = gsr.make_camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.near_z, cam.bg)
    keys = gsr.PARAM_GROUPS
    lrs = {"means": 1e-3, "scales": 5e-4, "quats": 2e-3, "opacities": 1e-2, "colors": 5e-3}
    rng = np.random.default_rng(3)
    m0 = {k: rng.normal(scale=1e-3, size=np.asarray(g[k]).shape).astype(np.float32) for k in keys}
    v0 = {k: rng.uniform(1e-8, 1e-6, size=np.asarray(g[k]).shape).astype(np.float32) for k in keys}
    poses = [np.asarray(pose, np.float32)[None], np.stack([np.asarray(pose, np.float32)] * 2)]
    poses[1][1, 4] += 0.02  # second view shifted 2 cm
    for pv in poses:
        runs = []
        for fused in (False, True):
            d = {k: v.clone() for k, v in G.to_dev(g).items()}
            m = {k: torch.from_numpy(m0[k]).cuda() for k in keys}
            v = {k: torch.from_numpy(v0[k]).cuda() for k in keys}
            pd = torch.from_numpy(pv).cuda()
            if pv.shape[0] == 1:
                c, dep, _, st = gsr.render_fwd(d["means"], d["scales"], d["quats"], d["opacities"], d["colors"],
                                               pd[0], camera)
            else:
                c, dep, _, st = gsr.render_fwd_batch(d["means"], d["scales"], d["quats"], d["opacities"],
                                                     d["colors"], pd, camera)
            gC = torch.full_like(c, 1e-3) * torch.sign(c - 0.3)
            gD = torch.full_like(dep, 1e-3) * torch.sign(dep - 1.0)
            if fused:
                gsr.render_bwd_adam(st, gC, gD, m, v, lrs, 3)
            else:
                gr = gsr.render_bwd(st, gC, gD, None, want_params=True, want_pose=False)
                gsr.adam_groups([d[k] for k in keys], [m[k] for k in keys], [v[k] for k in keys],
                                [gr[k] for k in keys], [lrs[k] for k in keys], 3)
            torch.cuda.synchronize()
            st.release()
            runs.append({k: (d[k].cpu().numpy(), m[k].cpu().numpy(), v[k].cpu().numpy()) for k in keys})
        sep, fus = runs
        for k in keys:
            moved = np.abs(sep[k][0] - np.asarray(g[k], np.float32)).max()
            assert moved > 0, k
            np.testing.assert_allclose(fus[k][0], sep[k][0], rtol=1e-6, atol=1e-7, err_msg=k)
            np.testing.assert_allclose(fus[k][1], sep[k][1], rtol=1e-4, atol=1e-12, err_msg=k)
            np.testing.assert_allclose(fus[k][2], sep[k][2], rtol=1e-4, atol=1e-15, err_msg=k)


def test_backward_fused_with_adam_rejects_other_parameters():
    """gsr_render_bwd_adam checks that the Adam parameters are the tensors the
    forward read (GSR_EINVAL otherwise) and that the step count is 1-based."""
    import ctypes
    torch = torch_()
    g, _, pose, cam = G.c1_case(0)
    out, st, d, pose_d = run_fwd(g, pose, cam)
    gC = torch.full((3, cam.height, cam.width), 1e-3, device="cuda")
    gD = torch.full((cam.height, cam.width), 1e-3, device="cuda")
    m = {k: torch.zeros_like(d[k]) for k in gsr.PARAM_GROUPS}
    v = {k: torch.zeros_like(d[k]) for k in gsr.PARAM_GROUPS}
    other = d["means"].clone()
    a = gsr.Adam5()
    for i, k in enumerate(gsr.PARAM_GROUPS):
        a.params[i] = (other if k == "means" else st.keep[i]).data_ptr()
        a.exp_avg[i] = m[k].data_ptr()
        a.exp_avg_sq[i] = v[k].data_ptr()
        a.lr[i] = 1e-3
    a.step, a.beta1, a.beta2, a.eps = 1, 0.9, 0.999, 1e-8
    lib, h = st.ctx.lib, st.ctx.h
    rc = lib.gsr_render_bwd_adam(h, st.h, ctypes.c_void_p(gC.data_ptr()), ctypes.c_void_p(gD.data_ptr()), None,
                                 ctypes.byref(a))
    assert rc != 0
    a.params[0] = st.keep[0].data_ptr()
    a.step = 0
    rc = lib.gsr_render_bwd_adam(h, st.h, ctypes.c_void_p(gC.data_ptr()), ctypes.c_void_p(gD.data_ptr()), None,
                                 ctypes.byref(a))
    assert rc != 0
    torch.cuda.synchronize()
    st.release()
