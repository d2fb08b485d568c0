"""Multi-keyframe mapping on the GPU: one sort and one compositing launch
(per-tile or persistent) for all views, against per-view renders and the
oracle; the tile-shape / blocks-per-CU autotuner."""
import numpy as np
import pytest

import oracle
from paper_2312_10070_amd import gsr, synth
from tests import gpu_cases as G
from tests import helpers as H

pytestmark = pytest.mark.gpu

CAM = synth.Intrinsics(200, 136, 100.0, 100.0, 100.0, 68.0)


def torch_():
    import torch
    return torch


def batch_scene(seed=0, n=40_000, V=4):
    torch = torch_()
    inp = synth.batched_inputs(seed, n, CAM, n_views=V, n_seed_views=6)
    g = {k: torch.from_numpy(v).cuda() for k, v in inp["gaussians"].items()}
    poses = torch.from_numpy(np.stack(inp["candidate_views"][:V])).cuda()
    return inp, g, poses


@pytest.mark.parametrize("bpc,shape", [(0, (16, 16)), (2, (16, 16)), (1, (8, 32)), (4, (32, 8))])
def test_batch_equals_sequential(bpc, shape):
    torch = torch_()
    inp, g, poses = batch_scene()
    cam = gsr.camera_from(CAM, bg=(0.1, 0.2, 0.3))
    opts = gsr.RasterOpts(tile_w=shape[0], tile_h=shape[1])
    args = (g["means"], g["scales"], g["quats"], g["opacities"], g["colors"])
    V = poses.shape[0]
    cb, db, ab, st = gsr.render_fwd_batch(*args, poses, cam, opts, blocks_per_cu=bpc)
    rng = np.random.default_rng(1)
    gC = torch.from_numpy((rng.normal(size=tuple(cb.shape)) * 1e-3).astype(np.float32)).cuda()
    gD = torch.from_numpy((rng.normal(size=tuple(db.shape)) * 1e-3).astype(np.float32)).cuda()
    out_b = gsr.render_bwd(st, gC, gD)
    sums = {k: torch.zeros_like(v) for k, v in g.items()}
    for v in range(V):
        c1, d1, a1, s1 = gsr.render_fwd(*args, poses[v].contiguous(), cam, opts)
        assert torch.equal(c1, cb[v]) and torch.equal(d1, db[v]) and torch.equal(a1, ab[v])
        o1 = gsr.render_bwd(s1, gC[v].contiguous(), gD[v].contiguous())
        for k in sums:
            sums[k] += o1[k]
        np.testing.assert_allclose(out_b["pose7"][v].cpu().numpy(), o1["pose7"].cpu().numpy(), rtol=1e-4,
                                   atol=1e-5 * float(o1["pose7"].abs().max()))
    torch.cuda.synchronize()
    for k in sums:
        a = out_b[k].cpu().numpy().astype(np.float64)
        b = sums[k].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-6 * np.abs(b).max())
    assert float(ab.mean()) > 0.05


def test_batch_matches_oracle():
    """Two posed views of the C1 scene, rendered in one batch, against the
    oracle view by view; parameter gradients against the oracle's sum."""
    torch = torch_()
    inp = synth.c1_inputs(0)
    cam = H.cam_of(synth.C1_CAMERA)
    p0 = np.array([1, 0, 0, 0, 0, 0, 0], np.float64)
    p1 = np.array([0.995, 0.03, -0.05, 0.02, 0.05, -0.03, 0.1]); p1[:4] /= np.linalg.norm(p1[:4])
    p1 = p1.astype(np.float32).astype(np.float64)
    g = G.certify(inp["gaussians"], p0, cam, 2e-4)
    g = G.certify(g, p1, cam, 2e-4)
    d = G.to_dev(g)
    poses = torch.tensor(np.stack([p0, p1]), dtype=torch.float32, device="cuda")
    camera = gsr.make_camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)
    cb, db, ab, st = gsr.render_fwd_batch(d["means"], d["scales"], d["quats"], d["opacities"], d["colors"], poses,
                                          camera, blocks_per_cu=2)
    rng = np.random.default_rng(3)
    gC = (rng.normal(size=(2, 3, 48, 64)) * 1e-3).astype(np.float32)
    gD = (rng.normal(size=(2, 48, 64)) * 1e-3).astype(np.float32)
    out = gsr.render_bwd(st, torch.from_numpy(gC).cuda(), torch.from_numpy(gD).cuda())
    torch.cuda.synchronize()
    refs = []
    for v, pose in enumerate((p0, p1)):
        opts = oracle.Opts(amb_rel=1e-4)
        orc = oracle.render(g, pose, cam, opts)
        G.compare_images(dict(color=cb[v].cpu().numpy(), depth=db[v].cpu().numpy(), alpha=ab[v].cpu().numpy()),
                         orc, {"color": 1e-4, "depth": 1e-4, "alpha": 1e-4})
        refs.append(oracle.backward(g, pose, cam, opts, gC[v].astype(np.float64), gD[v].astype(np.float64)))
        H.check_grad(f"pose{v}", out["pose7"][v].cpu().numpy(), refs[v]["grads"]["pose7"], refs[v]["aref"]["pose7"],
                     refs[v]["slack"]["pose7"], aref_plain=refs[v]["aref_plain"]["pose7"], case="batch 2 views")
    for k in ("means", "scales", "quats", "opacities", "colors"):
        ref = refs[0]["grads"][k] + refs[1]["grads"][k]
        aref = refs[0]["aref"][k] + refs[1]["aref"][k]
        aplain = refs[0]["aref_plain"][k] + refs[1]["aref_plain"][k]
        slack = refs[0]["slack"][k] + refs[1]["slack"][k]
        H.check_grad(k, out[k].cpu().numpy(), ref, aref, slack, aref_plain=aplain, case="batch 2 views")


def test_autotune_picks_a_timed_configuration():
    torch = torch_()
    inp, g, poses = batch_scene(1, n=30_000, V=3)
    cam = gsr.camera_from(CAM)
    args = (g["means"], g["scales"], g["quats"], g["opacities"], g["colors"])
    gC = torch.full((3, 3, CAM.height, CAM.width), 1e-3, device="cuda")
    gD = torch.full((3, CAM.height, CAM.width), 1e-3, device="cuda")
    best, bpc, table = gsr.autotune_batch(*args, poses, cam, gC, gD, reps=2)
    assert (best.tile_w, best.tile_h) in ((16, 16), (8, 32), (32, 8)) and bpc in (0, 1, 2, 4, 8)
    assert all(t > 0 for t in table.values())
    assert table[(best.tile_w, best.tile_h, bpc)] == min(table.values())
