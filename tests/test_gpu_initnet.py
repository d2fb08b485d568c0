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
            flat[off:off + 6 * initnet.HEAD_IN] = rng.normal(0, 0.2, 6 * initnet.HEAD_IN)
    net.set_params(torch.from_numpy(flat).cuda())
    x = torch.from_numpy(rng.uniform(0, 1, size=(B, 120, 160, 8)).astype(np.float32)).cuda().to(torch.bfloat16)
    net.set_input(x)
    return net, flat, x


def moment_pool(a4):
    """The head's pooled values from an NHWC last activation [B, 8, 10, 64]."""
    basis = oracle.moment_basis(a4.shape[1], a4.shape[2])
    return np.einsum("bhwc,khw->bkc", a4, basis).reshape(a4.shape[0], -1) / (a4.shape[1] * a4.shape[2])


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
    pool = moment_pool(acts[4])
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
    pool = moment_pool(acts[4])
    out = pool @ P["wfc"].T + P["bfc"]
    L, dout = oracle.initnet_loss(out, labels.cpu().numpy(), np.array(initnet.LABEL_SCALE))
    assert abs(loss.item() - L) <= 1e-4 * L
    np.testing.assert_allclose(g["wfc"], dout.T @ pool, rtol=1e-4, atol=1e-7)
    np.testing.assert_allclose(g["bfc"], dout.sum(0), rtol=1e-4, atol=1e-7)
    dpool = (dout @ P["wfc"]).reshape(B, 3, 64)
    basis = oracle.moment_basis(8, 10)
    ref_d4 = np.einsum("bkc,khw->bhwc", dpool, basis) / 80.0 * (acts[4] > 0)
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
    f64 = lambda a: a.astype(np.float64)
    ref = np.concatenate([pool(f64(rc)), pool(f64(rd))[None] * 0.25, 4 * pool(f64(oc) - f64(rc)),
                          4 * 0.25 * pool(f64(od) - f64(rd))[None]], 0).transpose(1, 2, 0)
    np.testing.assert_allclose(bf16_to_np(dst), ref, rtol=8e-3, atol=1e-6)


@pytest.fixture(scope="module")
def trained():
    """The network trained as the benchmark trains it: 50,000 pairs rendered at
    640 x 480 from procedural scenes built like tracking sub-maps, 15,000 Adam
    steps of batch 64; 1,024 held-out pairs from other scenes."""
    torch = torch_()
    cam = synth.TRACKING_CAMERA
    x, y = initnet.generate_pairs(50_000, seed=11, cam=cam)
    xv, yv = initnet.generate_pairs(1024, seed=12, cam=cam)
    net = gsr.InitNet(max_batch=64)
    net.set_params(torch.from_numpy(initnet.init_params(0)).cuda())
    losses = initnet.train(net, x, y, steps=15_000, batch=64, lr=2e-3)
    del x, y
    return net, losses, xv, yv


def test_training_reduces_loss(trained):
    net, losses, xv, yv = trained
    assert losses[-200:].mean() < 0.2 * losses[:20].mean(), (losses[:20].mean(), losses[-200:].mean())


def test_proposals_reduce_held_out_pose_error(trained):
    """On held-out scenes the predicted twist removes most of the perturbation:
    its mean squared (scaled) error is below 0.45 of the zero predictor's, and
    the rotation error left is under 0.6 degrees RMS per axis (from up to 3)."""
    torch = torch_()
    net, _, xv, yv = trained
    preds = torch.cat([initnet.predict(net, xv[i:i + 64]) for i in range(0, xv.shape[0], 64)]).cpu().numpy()
    y = yv.cpu().numpy()
    s = np.array(initnet.LABEL_SCALE)
    mse_pred = np.mean(((preds - y) / s) ** 2)
    mse_zero = np.mean((y / s) ** 2)
    rms = np.sqrt(np.mean((preds - y) ** 2, 0))
    print("held-out scaled MSE: network", mse_pred, "zero predictor", mse_zero, "RMS per axis", rms)
    assert mse_pred < 0.45 * mse_zero, (mse_pred, mse_zero)
    assert (np.rad2deg(rms[3:]) < 0.6).all(), rms


def test_learned_init_gain(trained):
    """Tracking frames at 640 x 480 with 500K Gaussians whose initial pose is
    off by 5 cm / 3 degrees: tracking from the network's proposal (up to three
    loss-judged steps) brings the camera within 1 mm / 0.1 degree of the
    ground truth on more frames than tracking from the initial pose does, and
    on the frames both reach it needs no more iterations on average."""
    torch = torch_()
    net, _, _, _ = trained
    budgets = (10, 20, 30, 40, 60, 80, 100)
    n_plain, n_learned, kept = [], [], []
    for frame in range(6):
        inp = synth.tracking_inputs(100 + frame, 500_000, trans_m=0.05, rot_deg=3.0)
        g = {k: torch.from_numpy(v).cuda() for k, v in inp["gaussians"].items()}
        args = (g["means"], g["scales"], g["quats"], g["opacities"], g["colors"])
        cam = gsr.camera_from(inp["camera"])
        gt = torch.from_numpy(inp["gt_pose7"]).cuda()
        oc, od, _, st = gsr.render_fwd(*args, gt, cam)
        st.release()
        init = torch.from_numpy(inp["init_pose7"]).cuda()
        kcap = tracking.overlap_capacity(*args, init, cam)
        graphs = {n: gsr.TrackGraph(*args, cam, oc, od, n_iters=n, K_cap=kcap) for n in budgets}

        def reached(n, start):
            q = start.clone()
            graphs[n].run(q)
            et, er = synth.pose_error(q.cpu().numpy(), inp["gt_pose7"])
            return et <= 1e-3 and er <= 0.1

        first = lambda start: next((n for n in budgets if reached(n, start)), None)
        n_plain.append(first(init))
        start, k, l0, l1 = initnet.propose(net, args, cam, oc, od, init, max_steps=3)
        kept.append(k)
        assert l1 <= l0
        n_learned.append(first(start))
        for tg in graphs.values():
            tg.close()
    print("iterations to 1 mm / 0.1 deg: plain", n_plain, "learned", n_learned, "proposal steps kept:", kept)
    reach_p = sum(n is not None for n in n_plain)
    reach_l = sum(n is not None for n in n_learned)
    assert sum(k > 0 for k in kept) >= 4, "the proposal should usually beat the initial pose"
    assert reach_l > reach_p, (n_plain, n_learned)
    both = [(p, l) for p, l in zip(n_plain, n_learned) if p is not None and l is not None]
    if both:
        assert np.mean([l for _, l in both]) <= np.mean([p for p, _ in both]), both
