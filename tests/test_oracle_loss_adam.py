"""Pins of the oracle's losses (Eq. 9, Eq. 10 L1 part, Eq. 15 with masks) and
its Adam step against numpy / torch library routines."""
import numpy as np
import torch

import oracle


def images(seed, P=(24, 32)):
    rng = np.random.default_rng(seed)
    Hh, Ww = P
    C = rng.uniform(0, 1, (3, Hh, Ww)).astype(np.float32)
    Ct = rng.uniform(0, 1, (3, Hh, Ww)).astype(np.float32)
    D = rng.uniform(0.5, 4, (Hh, Ww)).astype(np.float32)
    Dt = (D + rng.normal(0, 0.05, D.shape)).astype(np.float32)
    A = rng.uniform(0, 1, (Hh, Ww)).astype(np.float32)
    return C, D, A, Ct, Dt


def test_l1_loss_matches_numpy_and_signs():
    C, D, A, Ct, Dt = images(0)
    Ct[0, 0, 0] = C[0, 0, 0]  # an exact tie: sign(0) = 0
    L, gC, gD = oracle.loss_l1(C, D, Ct, Dt, 0.7, 1.3)
    P = D.size
    ref = 0.7 * np.abs(C.astype(np.float64) - Ct).mean() + 1.3 * np.abs(D.astype(np.float64) - Dt).mean()
    assert abs(L - ref) < 1e-12
    np.testing.assert_array_equal(gC, 0.7 * np.sign(C.astype(np.float64) - Ct) / (3 * P))
    np.testing.assert_array_equal(gD, 1.3 * np.sign(D.astype(np.float64) - Dt) / P)
    assert gC[0, 0, 0] == 0


def test_tracking_loss_median_mask_and_gradient():
    C, D, A, Ct, Dt = images(1)
    Dt[:3, :] = 0.0  # invalid observed depth
    D[5, 5] = Dt[5, 5] + 100.0  # a gross outlier
    r = oracle.loss_track(C, D, A, Ct, Dt, lambda_c=0.4, inlier_mult=50.0)
    valid = Dt > 0
    e = np.abs(D - Dt)  # float32 arithmetic, as the inputs carry
    ev = np.sort(e[valid])
    med = ev[(len(ev) - 1) // 2]
    assert r["median"] == med
    inl = valid & (e <= np.float32(50.0) * med)
    assert not inl[5, 5] and not inl[:3].any()
    assert r["n_inlier"] == int(inl.sum())
    w = np.where(inl, A.astype(np.float64) ** 3, 0.0)
    lc = np.abs(C.astype(np.float64) - Ct).sum(0)
    ld = np.abs(D.astype(np.float64) - Dt)
    assert abs(r["loss"] - (w * (0.4 * lc + 0.6 * ld)).sum()) < 1e-9
    np.testing.assert_allclose(r["gD"], w * (1 - 0.4) * np.sign(D.astype(np.float64) - Dt), rtol=1e-15, atol=0)
    np.testing.assert_allclose(r["gC"], w[None] * 0.4 * np.sign(C.astype(np.float64) - Ct), rtol=1e-15, atol=0)


def test_tracking_loss_median_even_count_lower_middle_and_empty():
    C, D, A, Ct, Dt = images(2, (2, 2))
    Dt[:] = 1.0
    D[:] = np.array([[1.1, 1.3], [1.2, 1.4]], np.float32)
    r = oracle.loss_track(C, D, A, Ct, Dt)
    assert r["median"] == np.float32(np.float32(1.2) - np.float32(1.0))
    Dt[:] = 0.0
    r = oracle.loss_track(C, D, A, Ct, Dt)
    assert r["n_inlier"] == 0 and r["loss"] == 0


def test_adam_matches_torch():
    rng = np.random.default_rng(0)
    p = rng.normal(size=7)
    m = np.zeros(7); v = np.zeros(7)
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 21):
        g = rng.normal(size=7)
        oracle.adam(p, m, v, g, step, 1e-3)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_const_velocity_pins():
    """Eq. 13: a pure translation extrapolates linearly; equal poses stay put;
    q and -q are the same rotation; a rotation by a then b about one axis
    extrapolates to (nearly) 2b - a for small steps."""
    from scipy.spatial.transform import Rotation
    p0 = np.array([1, 0, 0, 0, 0.1, 0.2, 0.3]); p1 = np.array([1, 0, 0, 0, 0.15, 0.1, 0.3])
    np.testing.assert_allclose(oracle.pose_const_velocity(p0, p1), [1, 0, 0, 0, 0.2, 0.0, 0.3], atol=1e-15)
    q = np.array([0.8, 0.2, -0.4, 0.4]); q /= np.linalg.norm(q)
    p = np.concatenate([q, [1, 2, 3]])
    np.testing.assert_allclose(oracle.pose_const_velocity(p, p), p, atol=1e-15)
    pm = p.copy(); pm[:4] *= -1
    np.testing.assert_allclose(oracle.pose_const_velocity(pm, p), p, atol=1e-15)
    axis = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    def qa(ang):
        x, y, z, w = Rotation.from_rotvec(axis * ang).as_quat()
        return np.array([w, x, y, z, 0, 0, 0])
    out = oracle.pose_const_velocity(qa(0.01), qa(0.02))
    ang = Rotation.from_quat([out[1], out[2], out[3], out[0]]).magnitude()
    assert abs(ang - 0.03) < 1e-6


def test_apply_twist_matches_scipy_and_inverts():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(4)
    for _ in range(10):
        q = rng.normal(size=4); q /= np.linalg.norm(q)
        p = np.concatenate([q, rng.normal(size=3)])
        xi = np.concatenate([rng.normal(0, 0.05, 3), rng.normal(0, 0.3, 3)])
        out = oracle.pose_apply_twist(p, xi)
        Rphi = Rotation.from_rotvec(xi[3:]).as_matrix()
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Ro = Rotation.from_quat([out[1], out[2], out[3], out[0]]).as_matrix()
        np.testing.assert_allclose(Ro, Rphi @ Rq, atol=1e-12)
        np.testing.assert_allclose(out[4:], Rphi @ p[4:] + xi[:3], atol=1e-12)
        # exp(-xi) undoes exp(xi) when rho is transported: T = exp(xi') exp(xi) T with xi' = (-Exp(-phi) rho, -phi)
        back = oracle.pose_apply_twist(out, np.concatenate([-(Rphi.T @ xi[:3]), -xi[3:]]))
        qb = back[:4] * np.sign(back[0]) ; qq = q * np.sign(q[0])
        np.testing.assert_allclose(qb, qq, atol=1e-12)
