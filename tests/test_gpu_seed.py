"""Seeding neighbour queries (Sec. 3.2 radius test, the supplement's
nearest-neighbour scale) on the HIP hash grid vs the oracle's brute force:
a minimum of FP32 distances and a comparison, so bit-exact."""
import numpy as np
import pytest

import oracle
from paper_2312_10070_amd import gsr

pytestmark = pytest.mark.gpu


def torch_():
    import torch
    return torch


def dev(a):
    torch = torch_()
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def run(p, q, rho, r_max):
    torch = torch_()
    nn, keep = gsr.seed_query(dev(p), dev(q), rho, r_max)
    torch.cuda.synchronize()
    return nn.cpu().numpy(), keep.cpu().numpy()


@pytest.mark.parametrize("n,m,rho,r_max", [(20000, 5003, 0.01, 0.05), (1, 7, 0.5, 0.5), (0, 100, 0.01, 0.02),
                                           (3000, 0, 0.01, 0.02), (50000, 4000, 0.002, 0.2)])
def test_seed_query_matches_oracle(n, m, rho, r_max):
    rng = np.random.default_rng(n + m)
    p = rng.uniform(-1.5, 1.5, (n, 3)).astype(np.float32)
    near = p[rng.integers(0, max(n, 1), m // 2)] + rng.normal(0, rho, (m // 2, 3)) if n else rng.normal(size=(m // 2, 3))
    q = np.concatenate([near, rng.uniform(-2, 2, (m - m // 2, 3))]).astype(np.float32)
    if n and m > 3:
        q[0] = p[0]           # distance 0: not kept
        q[1] = p[min(1, n - 1)] + np.float32(r_max) * 3  # beyond r_max
    nn_ref, keep_ref = oracle.seed_query(p, q, rho, r_max)
    nn, keep = run(p, q, rho, r_max)
    np.testing.assert_array_equal(nn, nn_ref)
    np.testing.assert_array_equal(keep, keep_ref)


def test_seed_query_room_scale_sampled():
    # sub-map of 500,000 means on the surfaces of a room (the mapping workload's
    # density), 100,000 candidates; the oracle checks a sample of 1,000
    from paper_2312_10070_amd import synth
    rng = np.random.default_rng(0)
    inp = synth.mapping_inputs(0, 500_000)
    p = inp["gaussians"]["means"].astype(np.float32)
    q = (p[rng.integers(0, len(p), 100_000)] + rng.normal(0, 0.01, (100_000, 3))).astype(np.float32)
    rho, r_max = 0.01, 0.1
    nn, keep = run(p, q, rho, r_max)
    idx = rng.choice(len(q), 1000, replace=False)
    nn_ref, keep_ref = oracle.seed_query(p, q[idx], rho, r_max)
    np.testing.assert_array_equal(nn[idx], nn_ref)
    np.testing.assert_array_equal(keep[idx], keep_ref)
    assert 0 < keep.sum() < len(q)


@pytest.mark.parametrize("offset", [0.0, -37.25, 300.0])
def test_seed_query_cell_boundaries(offset):
    """Means on the corners of the hash grid's cells (edge r_max (1 + 1e-3)),
    queries at just under r_max, exactly r_max and just over r_max from a mean
    along the axes and diagonals, near the origin and up to 300 m from it (cell
    coordinates near 6000): every mean within r_max lies in the 27 cells
    around the query whatever the rounding of the cell index, so the
    distances are exact."""
    r_max, rho = 0.05, 0.01
    h = r_max * 1.001
    k = np.arange(-3, 4)
    p = (offset + np.stack(np.meshgrid(k, k, k, indexing="ij"), -1).reshape(-1, 3) * h).astype(np.float32)
    dirs = np.array([[1, 0, 0], [0, -1, 0], [0, 0, 1], [1, 1, 0], [1, -1, 1], [-1, -1, -1]], np.float64)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    rng = np.random.default_rng(5)
    base = p[rng.choice(len(p), 40, replace=False)].astype(np.float64)
    q = np.concatenate([base[:, None] + s * r_max * dirs[None] for s in (1 - 1e-4, 1.0, 1 + 1e-4, 0.5, 0.1)])
    q = q.reshape(-1, 3).astype(np.float32)
    nn_ref, keep_ref = oracle.seed_query(p, q, rho, r_max)
    nn, keep = run(p, q, rho, r_max)
    np.testing.assert_array_equal(nn, nn_ref)
    np.testing.assert_array_equal(keep, keep_ref)
    cap = np.float32(np.float32(r_max) * np.float32(r_max))  # no mean within r_max
    assert (nn_ref < cap).any() and (nn_ref == cap).any()


def test_seed_query_bad_arguments():
    torch = torch_()
    p = dev(np.zeros((4, 3)))
    for rho, r_max in [(0.0, 1.0), (0.2, 0.1), (float("nan"), 1.0), (0.1, float("inf"))]:
        with pytest.raises(gsr.GsrError):
            gsr.seed_query(p, p, rho, r_max)
    with pytest.raises(ValueError):
        gsr.seed_query(dev(np.zeros((4, 2))), p, 0.1, 0.2)


def seed_frame(W, Hh, seed):
    from paper_2312_10070_amd import synth
    rng = np.random.default_rng(seed)
    cam_i = synth.Intrinsics(W, Hh, 0.9 * W, 0.9 * W, W / 2 + 0.3, Hh / 2 - 0.2)
    room = synth.make_room(seed)
    pose = synth.open_view(room, rng, synth.MAPPING_CAMERA)
    C, D = synth.render_frame(room, cam_i, pose)
    D[rng.uniform(size=D.shape) < 0.05] = 0.0  # holes in the observed depth
    A = rng.uniform(0, 1, D.shape).astype(np.float32)
    U = rng.uniform(0, 1, D.shape).astype(np.float32)
    return cam_i, np.asarray(pose, np.float32), C, D, A, U


@pytest.mark.parametrize("W,Hh,first", [(70, 45, True), (70, 45, False), (1200, 680, True), (1200, 680, False),
                                        (1, 1, True), (3, 200, True)])
def test_seed_candidates_match_oracle(W, Hh, first):
    torch = torch_()
    cam_i, pose, C, D, A, U = seed_frame(W, Hh, W + Hh)
    cam_o = oracle.Camera(W, Hh, cam_i.fx, cam_i.fy, np.float32(cam_i.cx), np.float32(cam_i.cy))
    pu, pg, thre = (0.05, 0.5, 0.05) if first else (0.3, 0.0, 0.0)
    P_ref, col_ref = oracle.seed_candidates(C, D, None if first else A, U, pose.astype(np.float64), cam_o, pu, pg,
                                            thre, 0.6)
    camera = gsr.camera_from(cam_i)
    pts, cols = gsr.seed_candidates(dev(C), dev(D), dev(U), dev(pose), camera, pu, pg, thre,
                                    alpha=None if first else dev(A), alpha_n=0.6)
    torch.cuda.synchronize()
    assert pts.shape[0] == len(P_ref)
    np.testing.assert_array_equal(cols.cpu().numpy(), col_ref.astype(np.float32))
    got = pts.cpu().numpy().astype(np.float64)
    scale = np.abs(P_ref).max() if len(P_ref) else 0.0
    np.testing.assert_allclose(got.reshape(-1, 3), P_ref.reshape(-1, 3), rtol=0, atol=2e-6 * (1 + scale))
    if W * Hh > 1000:
        assert 0 < len(P_ref) < W * Hh


@pytest.mark.parametrize("m,frac", [(5003, 0.3), (0, 0.0), (777, 1.0), (64, 0.0), (200000, 0.05)])
def test_seed_gaussians_match_oracle(m, frac):
    """New Gaussians (opacity 0.5, scale = the nearest-neighbour distance,
    identity rotation) from synthetic seeding outputs: bit-exact, including
    the correctly rounded square root."""
    torch = torch_()
    rng = np.random.default_rng(m + 3)
    pts = rng.uniform(-2, 2, (m, 3)).astype(np.float32)
    col = rng.uniform(0, 1, (m, 3)).astype(np.float32)
    nn = rng.uniform(1e-4, 2.5e-3, m).astype(np.float32)
    nn[: m // 7] = np.float32(0.05) * np.float32(0.05)  # no neighbour within r_max
    keep = (rng.uniform(size=m) < frac).astype(np.int32)
    ref = oracle.seed_gaussians(pts, col, nn, keep)
    got = gsr.seed_gaussians(dev(pts), dev(col), dev(nn), torch.from_numpy(keep).cuda())
    torch.cuda.synchronize()
    for k in ("means", "scales", "quats", "opacities", "colors"):
        np.testing.assert_array_equal(got[k].cpu().numpy(), ref[k], err_msg=k)


def test_seed_pipeline_adds_gaussians_where_the_submap_is_empty():
    """Candidates -> neighbour queries -> new Gaussians, each call checked
    against the oracle on the same inputs; the new Gaussians sit only where
    the sub-map had none within rho."""
    torch = torch_()
    rng = np.random.default_rng(21)
    sub = rng.uniform(-0.5, 0.5, (4000, 3)).astype(np.float32)
    pts = np.concatenate([sub[:1500] + rng.normal(0, 0.002, (1500, 3)),
                          rng.uniform(-0.6, 0.6, (1500, 3))]).astype(np.float32)
    col = rng.uniform(0, 1, (3000, 3)).astype(np.float32)
    rho, r_max = 0.01, 0.05
    nn, keep = gsr.seed_query(dev(sub), dev(pts), rho, r_max)
    nn_ref, keep_ref = oracle.seed_query(sub, pts, rho, r_max)
    np.testing.assert_array_equal(nn.cpu().numpy(), nn_ref)
    np.testing.assert_array_equal(keep.cpu().numpy(), keep_ref)
    g = gsr.seed_gaussians(dev(pts), dev(col), nn, keep)
    ref = oracle.seed_gaussians(pts, col, nn_ref, keep_ref)
    for k in ref:
        np.testing.assert_array_equal(g[k].cpu().numpy(), ref[k], err_msg=k)
    # every new mean is at least rho from every sub-map mean
    d2, _ = oracle.seed_query(sub, ref["means"], rho, r_max)
    assert (d2 >= np.float32(rho) * np.float32(rho)).all()
