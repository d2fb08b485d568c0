"""Tracking path at its full size (640 x 480, 500K Gaussians), against the
oracle: the pose-only backward the tracking graph runs (the six-field
compositing reduction, no opacity or colour gradients) driven by the real
Eq. 15 upstream gradients on sampled pixels, and the Eq. 15 loss with the
supplement's masks (exact median by radix select) on the whole frame.
Sec. 3.4, Eq. 14-15."""
import numpy as np
import pytest

import oracle
from paper_2312_10070_amd import gsr, synth
from tests import helpers as H

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(300)]

# as in the full-size mapping test: FP32 screen positions far off-centre carry
# ~1e-4 px of rounding, FP32 camera depths ~3e-7 relative
OPTS = oracle.Opts(amb_rel=2e-4, amb_z=5e-7)


@pytest.fixture(scope="module")
def frame():
    import torch
    inp = synth.tracking_inputs(0, 500_000)
    cam = gsr.camera_from(inp["camera"])
    g = {k: torch.from_numpy(v).cuda() for k, v in inp["gaussians"].items()}
    args = (g["means"], g["scales"], g["quats"], g["opacities"], g["colors"])
    obs_c, obs_d, _, st = gsr.render_fwd(*args, torch.from_numpy(inp["gt_pose7"]).cuda(), cam)
    st.release()
    return inp, cam, args, obs_c.clone(), obs_d.clone()


def test_pose_backward_fullsize_matches_oracle(frame):
    """The tracking iteration's backward (want_params=False: the six-field
    reduction) at the initial pose; upstream = the GPU's Eq. 15 gradients on
    600 sampled pixels (zero elsewhere), the same FP32 arrays on both sides."""
    import torch
    inp, cam, args, obs_c, obs_d = frame
    pose = inp["init_pose7"]
    color, depth, alpha, st = gsr.render_fwd(*args, torch.from_numpy(pose).cuda(), cam)
    _, gC_full, gD_full, _ = gsr.loss_track(color, depth, alpha, obs_c, obs_d, 0.5, 50.0)
    torch.cuda.synchronize()
    W, Hh = cam.width, cam.height
    rng = np.random.default_rng(11)
    pixels = np.sort(rng.choice(W * Hh, 600, replace=False))
    yy, xx = pixels // W, pixels % W
    gC = np.zeros((3, Hh, W), np.float32)
    gD = np.zeros((Hh, W), np.float32)
    gC[:, yy, xx] = gC_full.cpu().numpy()[:, yy, xx]
    gD[yy, xx] = gD_full.cpu().numpy()[yy, xx]
    assert np.count_nonzero(gD) > 300  # most sampled pixels are inliers with a residual
    out = gsr.render_bwd(st, torch.from_numpy(gC).cuda(), torch.from_numpy(gD).cuda(), None, want_params=False,
                         want_pose=True)
    torch.cuda.synchronize()
    st.release()
    ocam = H.cam_of(inp["camera"])
    ref = oracle.backward(inp["gaussians"], pose.astype(np.float64), ocam, OPTS, gC.astype(np.float64),
                          gD.astype(np.float64), pixels=pixels, nthreads=8)
    assert ref["n_unverifiable"] <= 0.02 * len(pixels)
    for k in ("pose7", "twist6"):
        H.check_grad_ref(k, out[k].cpu().numpy().astype(np.float64), ref, case="full-size tracking six-field")
    # the translation part of the twist is the translation gradient (left perturbation)
    np.testing.assert_allclose(out["twist6"].cpu().numpy()[:3], out["pose7"].cpu().numpy()[4:], rtol=1e-6,
                               atol=1e-12)


@pytest.mark.parametrize("variant", ["rendered", "holes_quantised"])
def test_loss_track_fullsize_matches_oracle(frame, variant):
    """Eq. 15 on the whole 640 x 480 frame: the median is an exact element
    (compared bit for bit), the inlier and alpha^3 masks, the loss and its
    upstream gradients per element. 'holes_quantised' zeroes 20 % of the
    observed depths (invalid pixels) and rounds the rest to 1 mm, so the depth
    errors carry many exact ties around the median."""
    import torch
    inp, cam, args, obs_c, obs_d = frame
    color, depth, alpha, st = gsr.render_fwd(*args, torch.from_numpy(inp["init_pose7"]).cuda(), cam)
    st.release()
    od = obs_d.cpu().numpy().copy()
    if variant == "holes_quantised":
        rng = np.random.default_rng(3)
        od = (np.round(od * 1000.0) / 1000.0).astype(np.float32)
        od[rng.uniform(size=od.shape) < 0.2] = 0.0
    od_dev = torch.from_numpy(od).cuda()
    loss, gC, gD, med = gsr.loss_track(color, depth, alpha, obs_c, od_dev, 0.5, 50.0)
    torch.cuda.synchronize()
    C, D, A = color.cpu().numpy(), depth.cpu().numpy(), alpha.cpu().numpy()
    r = oracle.loss_track(C, D, A, obs_c.cpu().numpy(), od, 0.5, 50.0)
    assert med.item() == r["median"]
    assert r["n_inlier"] > 0.5 * (od > 0).sum()
    assert abs(loss.item() - r["loss"]) <= 1e-5 * abs(r["loss"])
    np.testing.assert_allclose(gC.cpu().numpy(), r["gC"], rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(gD.cpu().numpy(), r["gD"], rtol=1e-5, atol=1e-9)
