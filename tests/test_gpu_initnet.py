"""The BF16 MFMA tracking-initialisation CNN against the FP64 oracle, its
training on renderer-generated pairs, and what it gains for tracking.

Layer checks feed the oracle the same BF16 values the GPU consumed (the
previous layer's BF16 output read back), so the only differences are FP32
accumulation order and the BF16 rounding of each output: relative 1e-2 of
the layer's RMS plus 1e-2 of each value."""
import numpy as np
import pytest

import oracle
from paper_2312_10070_amd import gsr, initnet, synth, tracking

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

SHAPES = [(120, 160, 8), (60, 80, 64), (30, 40, 64), (15, 20, 64), (8, 10, 64)]


def torch_():
    import torch
    return torch


def bf16_to_np(t):
    return t.float().cpu().numpy().astype(np.float64)


def nhwc_to_nchw(a):
    return a.transpose(0, 3, 1, 2)


def close(name, got, ref, rel=1e-2, rms_frac=1e-2):
    rms = np.sqrt(np.mean(ref ** 2)) + 1e-30
    err = np.abs(got - ref)
    tol = rel * np.abs(ref) + rms_frac * rms
    bad = err > tol
    assert not bad.any(), f"{name}: {int(bad.sum())} of {bad.size} out of tolerance, worst err {err.max():.3g} rms {rms:.3g}"


def setup_net(B=3, seed=0):
    torch = torch_()
    net = gsr.InitNet(max_batch=8)
    flat = initnet.init_params(seed)
    # non-zero biases so the bias paths are exercised
    lay, _ = initnet.layout()
    rng = np.random.default_rng(seed)
    for name, shape, off in lay:
        if name.startswith("b"):
            flat[off:off + shape[0]] = rng.normal(0, 0.05, shape[0])
        if name == "wfc":
            flat[off:off + 6 * 64] = rng.normal(0, 0.2, 6 * 64)
    net.set_params(torch.from_numpy(flat).cuda())
    x = torch.from_numpy(rng.uniform(0, 1, size=(B, 120, 160, 8)).astype(np.float32)).cuda().to(torch.bfloat16)
    net.set_input(x)
    return net, flat, x


def test_layers_forward_match_oracle():
    torch = torch_()
    B = 3
    net, flat, x = setup_net(B)
    out = net.forward(B)
    torch.cuda.synchronize()
    P = initnet.to_oihw(flat.astype(np.float32).astype(np.float64))
    # weights as the GPU uses them: BF16-rounded
    Pb = initnet.to_oihw(torch.from_numpy(flat).to(torch.bfloat16).float().numpy())
    acts = [bf16_to_np(net.activation(l, B, SHAPES[l])[0]) for l in range(5)]
    for l in range(4):
        ref = np.maximum(oracle.conv2d(nhwc_to_nchw(acts[l]), Pb[f"w{l}"], P[f"b{l}"]), 0.0)
        close(f"layer{l}", nhwc_to_nchw(acts[l + 1]), ref)
    pool = acts[4].mean(axis=(1, 2))
    ref_out = pool @ P["wfc"].T + P["bfc"]
    np.testing.assert_allclose(out.cpu().numpy(), ref_out, rtol=1e-4, atol=1e-5)


def test_layers_backward_match_oracle():
    torch = torch_()
    B = 3
    net, flat, x = setup_net(B, seed=1)
    net.forward(B)
    rng = np.random.default_rng(2)
    labels = torch.from_numpy(rng.normal(0, 0.02, (B, 6)).astype(np.float32)).cuda()
    scale = torch.tensor(initnet.LABEL_SCALE, device="cuda")
    loss = net.backward(B, labels, scale)
    _, grads = net.get_params(with_grads=True)
    torch.cuda.synchronize()
    g = initnet.to_oihw(grads.cpu().numpy().astype(np.float64))
    Pb = initnet.to_oihw(torch.from_numpy(flat).to(torch.bfloat16).float().numpy())
    P = initnet.to_oihw(flat.astype(np.float64))
    acts, dacts = [], []
    for l in range(5):
        a, d = net.activation(l, B, SHAPES[l])
        acts.append(bf16_to_np(a)); dacts.append(bf16_to_np(d))
    # head and loss, from the GPU's own last activation
    pool = acts[4].mean(axis=(1, 2))
    out = pool @ P["wfc"].T + P["bfc"]
    L, dout = oracle.initnet_loss(out, labels.cpu().numpy(), np.array(initnet.LABEL_SCALE))
    assert abs(loss.item() - L) <= 1e-4 * L
    np.testing.assert_allclose(g["wfc"], dout.T @ pool, rtol=1e-4, atol=1e-7)
    np.testing.assert_allclose(g["bfc"], dout.sum(0), rtol=1e-4, atol=1e-7)
    dpool = dout @ P["wfc"]
    ref_d4 = np.broadcast_to(dpool[:, None, None, :] / 80.0, acts[4].shape) * (acts[4] > 0)
    close("dact4", dacts[4], ref_d4)
    for l in range(3, -1, -1):
        dy = nhwc_to_nchw(dacts[l + 1])
        dx, dw, db = oracle.conv2d_bwd(nhwc_to_nchw(acts[l]), Pb[f"w{l}"], dy, want_dx=l > 0)
        close(f"dW{l}", g[f"w{l}"], dw, rel=2e-3, rms_frac=2e-3)
        close(f"db{l}", g[f"b{l}"], db, rel=2e-3, rms_frac=2e-3)
        if l > 0:
            close(f"dact{l}", nhwc_to_nchw(dacts[l]), dx * (nhwc_to_nchw(acts[l]) > 0))


def test_pack_input_matches_average_pooling():
    torch = torch_()
    rng = np.random.default_rng(3)
    rc = rng.uniform(0, 1, (3, 240, 320)).astype(np.float32); rd = rng.uniform(0.5, 5, (240, 320)).astype(np.float32)
    oc = rng.uniform(0, 1, (3, 240, 320)).astype(np.float32); od = rng.uniform(0.5, 5, (240, 320)).astype(np.float32)
    dst = torch.empty((120, 160, 8), device="cuda", dtype=torch.bfloat16)
    dev = lambda a: torch.from_numpy(a).cuda()
    gsr.pack_rgbd_pair(dev(rc), dev(rd), dev(oc), dev(od), dst, 0.25)
    pool = lambda a: a.reshape(a.shape[:-2] + (120, 2, 160, 2)).mean(axis=(-3, -1))
    ref = np.concatenate([pool(rc), pool(rd)[None] * 0.25, pool(oc), pool(od)[None] * 0.25], 0).transpose(1, 2, 0)
    np.testing.assert_allclose(bf16_to_np(dst), ref, rtol=8e-3, atol=1e-6)


CAM = synth.Intrinsics(320, 240, 262.5, 262.5, 160.0, 120.0)


@pytest.fixture(scope="module")
def trained():
    torch = torch_()
    x, y = initnet.generate_pairs(32768, seed=11, cam=CAM)
    xv, yv = initnet.generate_pairs(512, seed=12, cam=CAM)
    net = gsr.InitNet(max_batch=64)
    net.set_params(torch.from_numpy(initnet.init_params(0)).cuda())
    losses = initnet.train(net, x, y, steps=8000, batch=64, lr=2e-3)
    del x, y
    return net, losses, xv, yv


def test_training_reduces_loss(trained):
    net, losses, xv, yv = trained
    assert losses[-100:].mean() < 0.5 * losses[:20].mean(), (losses[:20].mean(), losses[-100:].mean())


def test_proposals_reduce_held_out_pose_error(trained):
    """On held-out rooms the predicted twist removes a clear part of the
    perturbation: its mean squared (scaled) error is below 0.6 of the zero
    predictor's. A global-average-pooled network cannot undo every
    rotation/translation ambiguity, so the bar is a clear gain, not a fit."""
    torch = torch_()
    net, _, xv, yv = trained
    preds = torch.cat([initnet.predict(net, xv[i:i + 64]) for i in range(0, xv.shape[0], 64)]).cpu().numpy()
    y = yv.cpu().numpy()
    s = np.array(initnet.LABEL_SCALE)
    mse_pred = np.mean(((preds - y) / s) ** 2)
    mse_zero = np.mean((y / s) ** 2)
    print("held-out scaled MSE: network", mse_pred, "zero predictor", mse_zero)
    assert mse_pred < 0.6 * mse_zero, (mse_pred, mse_zero)


def test_learned_init_gain(trained):
    """On frames perturbed by 5 cm / 3 degrees (the training range), tracking
    from the network's proposal (kept only when Eq. 15 prefers it)
    reaches the accuracy of 100 plain iterations (their final error + 5 %, at
    least 0.5 mm) in fewer iterations, on average, than plain tracking does."""
    torch = torch_()
    net, _, _, _ = trained
    budgets = (10, 15, 20, 30, 40, 50, 60, 80, 100)
    n_plain, n_learned, used = [], [], 0
    for frame in range(8):
        inp = synth.tracking_inputs(100 + frame, 60_000, CAM, n_views=3, trans_m=0.05, rot_deg=3.0)
        g = {k: torch.from_numpy(v).cuda() for k, v in inp["gaussians"].items()}
        args = (g["means"], g["scales"], g["quats"], g["opacities"], g["colors"])
        cam = gsr.camera_from(CAM)
        gt = torch.from_numpy(inp["gt_pose7"]).cuda()
        oc, od, _, st = gsr.render_fwd(*args, gt, cam)
        st.release()
        init = torch.from_numpy(inp["init_pose7"]).cuda()
        kcap = tracking.overlap_capacity(*args, init, cam)
        graphs = {n: gsr.TrackGraph(*args, cam, oc, od, n_iters=n, K_cap=kcap) for n in budgets}

        def err_after(n, start):
            q = start.clone()
            graphs[n].run(q)
            return synth.pose_error(q.cpu().numpy(), inp["gt_pose7"])[0]

        thr = max(1.05 * err_after(100, init), 5e-4)
        first = lambda start: next((n for n in budgets if err_after(n, start) <= thr), 101)
        n_plain.append(first(init))
        start, use, l0, l1 = initnet.propose(net, args, cam, oc, od, init)
        used += use
        n_learned.append(first(start))
        for tg in graphs.values():
            tg.close()
    print("iterations to the target error: plain", n_plain, "learned", n_learned, "proposals used:", used)
    assert used >= 4, "the proposal should usually beat the initial pose"
    assert np.mean(n_learned) < np.mean(n_plain), (n_plain, n_learned)
