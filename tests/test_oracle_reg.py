"""Pins of the oracle's isotropic scale regulariser (Eq. 11; sbar_k = the mean of
Gaussian k's own three scales) against hand-derived values, invariances and
finite differences."""
import numpy as np

import oracle


def test_closed_forms():
    s = np.array([[1.0, 2.0, 3.0], [1.0, 1.0, 4.0], [2.0, 2.0, 2.0], [0.5, 0.2, 0.2]])
    L, g = oracle.loss_reg(s)
    # |r| sums: (1, 0, 1) -> 2; (1, 1, 2) -> 4; 0; sbar = 0.3: (0.2, 0.1, 0.1) -> 0.4
    assert abs(L - (2 + 4 + 0 + 0.4) / 4) < 1e-15
    ref = np.array([[-1, 0, 1], [-2 / 3, -2 / 3, 4 / 3], [0, 0, 0], [4 / 3, -2 / 3, -2 / 3]]) / 4
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-15)


def test_isotropic_is_zero_and_empty():
    # dyadic scales, so that (a + a + a) / 3 == a exactly and every r is 0
    s = np.repeat(np.random.default_rng(0).integers(1, 64, (50, 1)) / 64.0, 3, axis=1)
    L, g = oracle.loss_reg(s)
    assert L == 0.0 and not g.any()
    # any isotropic scales: only the rounding of sbar remains
    s = np.repeat(np.random.default_rng(0).uniform(0.01, 1, (50, 1)), 3, axis=1)
    assert oracle.loss_reg(s)[0] < 1e-15
    L, g = oracle.loss_reg(np.zeros((0, 3)))
    assert L == 0.0 and g.shape == (0, 3)


def test_homogeneous_and_axis_symmetric():
    rng = np.random.default_rng(1)
    s = np.exp(rng.normal(-3, 0.3, (200, 3)))
    L, g = oracle.loss_reg(s)
    L2, g2 = oracle.loss_reg(2.5 * s)
    assert abs(L2 - 2.5 * L) < 1e-15 * max(1, L2) * 10
    np.testing.assert_array_equal(g2, g)
    perm = [2, 0, 1]
    L3, g3 = oracle.loss_reg(s[:, perm])
    assert abs(L3 - L) < 1e-15
    np.testing.assert_array_equal(g3, g[:, perm])


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    s = np.exp(rng.normal(-3, 0.3, (40, 3)))
    _, g = oracle.loss_reg(s)
    h = 1e-9
    fd = np.empty_like(s)
    for i in np.ndindex(s.shape):
        sp = s.copy(); sp[i] += h
        sm = s.copy(); sm[i] -= h
        fd[i] = (oracle.loss_reg(sp)[0] - oracle.loss_reg(sm)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=0, atol=1e-6 * np.abs(fd).max())


def test_prune_definition():
    # supplement: Gaussians with opacity below the threshold are removed
    o = np.array([0.05, 0.1, 0.5, np.nan, 0.0999999, 1.0], np.float32)
    means = np.arange(18, dtype=np.float32).reshape(6, 3)
    n, (kept,) = oracle.prune([{"opacities": o, "means": means}], 0.1)
    assert n == 3
    np.testing.assert_array_equal(kept["opacities"], np.array([0.1, 0.5, 1.0], np.float32))
    np.testing.assert_array_equal(kept["means"], means[[1, 2, 5]])
    n2, (again,) = oracle.prune([kept], 0.1)  # idempotent
    assert n2 == 3 and all(np.array_equal(again[k], kept[k]) for k in kept)
    assert oracle.prune([{"opacities": o}], float("inf"))[0] == 0
    assert oracle.prune([{"opacities": o}], -float("inf"))[0] == 5  # NaN still removed


def test_seed_query_definition():
    # Sec. 3.2 radius test and the supplement's nearest-neighbour distance
    p = np.array([[0, 0, 0], [1, 0, 0], [0, 0.5, 0]], np.float32)
    q = np.array([[0.1, 0, 0], [0, 0.5, 0.004], [5, 5, 5], [0.5, 0.25, 0]], np.float32)
    nn, keep = oracle.seed_query(p, q, rho=0.01, r_max=0.3)
    np.testing.assert_allclose(nn, [0.01, 0.004 ** 2, 0.09, 0.09], rtol=1e-6)
    np.testing.assert_array_equal(keep, [1, 0, 1, 1])
    nn0, keep0 = oracle.seed_query(np.zeros((0, 3)), q, 0.01, 0.3)
    assert (nn0 == np.float32(0.3) * np.float32(0.3)).all() and keep0.all()


def test_seed_query_matches_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(5)
    p = rng.uniform(-1, 1, (3000, 3)).astype(np.float32)
    q = np.concatenate([p[:500] + rng.normal(0, 0.01, (500, 3)), rng.uniform(-1.2, 1.2, (500, 3))]).astype(np.float32)
    r_max = 0.08
    nn, keep = oracle.seed_query(p, q, 0.02, r_max)
    d, _ = cKDTree(p.astype(np.float64)).query(q.astype(np.float64))
    ref = np.minimum(d, r_max)
    np.testing.assert_allclose(np.sqrt(nn.astype(np.float64)), ref, rtol=1e-6, atol=1e-7)
    clear = np.abs(d - 0.02) > 1e-6
    np.testing.assert_array_equal(keep[clear], (d[clear] >= 0.02).astype(np.int32))
    perm = rng.permutation(len(p))  # order of the means does not matter
    nn2, _ = oracle.seed_query(p[perm], q, 0.02, r_max)
    np.testing.assert_array_equal(nn2, nn)


def test_seed_gaussians_definition():
    # supplement: a new Gaussian's opacity starts at 0.5 and its scale at the
    # nearest-neighbour distance in the active sub-map (checked against a k-d
    # tree, independent of the oracle's own distance computation); Sec. 3.2:
    # only the points with no neighbour within rho are added, in their order
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(11)
    p = rng.uniform(-1, 1, (2000, 3)).astype(np.float32)
    q = np.concatenate([p[:300] + rng.normal(0, 0.004, (300, 3)), rng.uniform(-1.1, 1.1, (700, 3))]).astype(np.float32)
    col = rng.uniform(0, 1, (1000, 3)).astype(np.float32)
    rho, r_max = 0.01, 0.05
    nn, keep = oracle.seed_query(p, q, rho, r_max)
    g = oracle.seed_gaussians(q, col, nn, keep)
    d, _ = cKDTree(p.astype(np.float64)).query(q.astype(np.float64))
    sel = np.flatnonzero(keep)
    assert len(sel) == g["means"].shape[0] and 0 < len(sel) < 1000
    clear = np.abs(d - rho) > 1e-6
    np.testing.assert_array_equal(keep[clear], (d[clear] >= rho).astype(np.int32))
    np.testing.assert_allclose(g["scales"], np.repeat(np.minimum(d[sel], r_max)[:, None], 3, 1), rtol=1e-6)
    assert (g["scales"] >= np.float32(rho) * (1 - 1e-6)).all()
    np.testing.assert_array_equal(g["opacities"], np.full(len(sel), 0.5, np.float32))
    np.testing.assert_array_equal(g["quats"], np.tile(np.array([1, 0, 0, 0], np.float32), (len(sel), 1)))
    np.testing.assert_array_equal(g["means"], q[sel])
    np.testing.assert_array_equal(g["colors"], col[sel])
    empty = oracle.seed_gaussians(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.int32))
    assert all(v.shape[0] == 0 for v in empty.values())


def test_seed_candidates_definition():
    from scipy.spatial.transform import Rotation
    cam = oracle.Camera(4, 3, 2.0, 2.5, 1.5, 1.0)
    D = np.array([[1, 2, 0, 1], [1, 1, 3, 1], [2, 1, 1, 1]], np.float32)
    C = np.zeros((3, 3, 4), np.float32)
    ident = np.array([1, 0, 0, 0, 0, 0, 0.0])
    # p = 1: every pixel with depth; back-projection by the pinhole model
    P, _ = oracle.seed_candidates(C, D, None, np.zeros((3, 4)), ident, cam, 1.0)
    assert len(P) == 11
    np.testing.assert_allclose(P[0], [(0 - 1.5) * 1 / 2.0, (0 - 1.0) * 1 / 2.5, 1.0])
    np.testing.assert_allclose(P[1], [(1 - 1.5) * 2 / 2.0, (0 - 1.0) * 2 / 2.5, 2.0])
    # p = 0 and the alpha mask
    assert len(oracle.seed_candidates(C, D, None, np.full((3, 4), 0.5), ident, cam, 0.0)[0]) == 0
    A = np.full((3, 4), 0.9, np.float32); A[1, 1] = 0.5
    P, _ = oracle.seed_candidates(C, D, A, np.zeros((3, 4)), ident, cam, 1.0)
    np.testing.assert_allclose(P, [[(1 - 1.5) * 1 / 2.0, 0.0, 1.0]])
    # a posed camera: the points project back to their pixels and depths
    rng = np.random.default_rng(0)
    q = rng.normal(size=4); q /= np.linalg.norm(q)
    pose = np.concatenate([q, [0.3, -0.2, 1.0]])
    P, _ = oracle.seed_candidates(C, D, None, np.zeros((3, 4)), pose, cam, 1.0)
    Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    Xc = P @ Rm.T + pose[4:]
    ys, xs = np.nonzero(D > 0)
    np.testing.assert_allclose(Xc[:, 2], D[ys, xs], atol=1e-12)
    np.testing.assert_allclose(cam.fx * Xc[:, 0] / Xc[:, 2] + cam.cx, xs, atol=1e-12)
    np.testing.assert_allclose(cam.fy * Xc[:, 1] / Xc[:, 2] + cam.cy, ys, atol=1e-12)


def test_seed_candidates_colour_gradient():
    # a vertical step edge: only the interior pixels next to it have a gradient
    cam = oracle.Camera(6, 5, 3.0, 3.0, 3.0, 2.5)
    C = np.zeros((3, 5, 6), np.float32); C[:, :, 3:] = 0.9
    D = np.ones((5, 6), np.float32)
    P, col = oracle.seed_candidates(C, D, None, np.full((5, 6), 0.5), np.array([1, 0, 0, 0, 0, 0, 0.0]), cam,
                                    0.0, 1.0, grad_thre=0.5)
    xs = np.round(P[:, 0] / P[:, 2] * cam.fx + cam.cx).astype(int)
    ys = np.round(P[:, 1] / P[:, 2] * cam.fy + cam.cy).astype(int)
    assert sorted(zip(ys.tolist(), xs.tolist())) == [(y, x) for y in (1, 2, 3) for x in (2, 3)]
    np.testing.assert_allclose(col[xs == 3], 0.9, atol=1e-7)


def test_submap_trigger_definition():
    from scipy.spatial.transform import Rotation
    I = np.array([1, 0, 0, 0, 0, 0, 0.0])
    assert oracle.submap_trigger(I, [1, 0, 0, 0, 0.6, 0, 0])
    assert not oracle.submap_trigger(I, [1, 0, 0, 0, 0.4, 0, 0])

    def rot(deg, axis, t=(0, 0, 0)):
        q = Rotation.from_rotvec(np.deg2rad(deg) * np.asarray(axis, float)).as_quat()  # x, y, z, w
        return np.concatenate([[q[3], q[0], q[1], q[2]], t])

    assert oracle.submap_trigger(I, rot(60, [0, 1, 0]))
    assert not oracle.submap_trigger(I, rot(40, [1, 1, 0] / np.sqrt(2)))
    assert not oracle.submap_trigger(rot(10, [0, 0, 1]), rot(-10, [0, 0, 1]))  # 20 degrees apart
    # same t, but a 40-degree turn moves the camera centre c = -R^T t by 2 sin(20 deg) |t| = 0.68 m
    t = (1.0, 0.0, 0.0)
    assert oracle.submap_trigger(rot(0, [0, 1, 0], t), rot(40, [0, 1, 0], t))
    # a 40-degree turn about the camera centre: t changes, the centre does not
    Rm = Rotation.from_rotvec(np.deg2rad(40) * np.array([0, 1, 0])).as_matrix()
    c = np.array([2.0, 0.5, -1.0])
    assert not oracle.submap_trigger(np.concatenate([[1, 0, 0, 0], -c]), rot(40, [0, 1, 0], -Rm @ c))


def test_merge_definition():
    g = {"means": np.array([[0, 0, 0], [1, 0, 0]], np.float32), "opacities": np.array([0.5, 0.6], np.float32)}
    s = {"means": np.array([[0.005, 0, 0], [0.5, 0, 0], [1, 0.02, 0]], np.float32),
         "opacities": np.array([0.1, 0.2, 0.3], np.float32)}
    m = oracle.merge_submap(g, s, rho=0.01)
    np.testing.assert_array_equal(m["means"], np.concatenate([g["means"], s["means"][1:]]))
    np.testing.assert_array_equal(m["opacities"], np.array([0.5, 0.6, 0.2, 0.3], np.float32))
