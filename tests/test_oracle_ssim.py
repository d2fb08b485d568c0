"""Pins of the oracle's SSIM term of the mapping colour loss (Eq. 10, SSIM after
Wang et al. 2004 with its standard 11x11, sigma 1.5 Gaussian window, zero
padding, C1 = 1e-4, C2 = 9e-4) against closed forms, a library filter and
finite differences."""
import numpy as np
import pytest
from scipy import ndimage
from scipy.signal import windows

import oracle

C1, C2 = 1e-4, 9e-4


def pair(seed, shape=(3, 19, 23)):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, shape)
    Y = np.clip(X + rng.normal(0, 0.15, shape), 0, 1)
    return X, Y


def test_identical_images_give_one_and_zero_gradient():
    X, _ = pair(0)
    mean, mp, g = oracle.ssim(X, X)
    assert abs(mean - 1.0) < 1e-12
    np.testing.assert_allclose(mp, 1.0, atol=1e-12)
    assert np.abs(g).max() < 1e-15


def test_constant_images_interior_closed_form():
    # away from the border every window sees one value: no variance, so only
    # the luminance factor (2ab + C1) / (a^2 + b^2 + C1) remains
    a, b = 0.3, 0.7
    X = np.full((1, 23, 25), a)
    Y = np.full((1, 23, 25), b)
    _, mp, _ = oracle.ssim(X, Y, want_grad=False)
    ref = (2 * a * b + C1) / (a * a + b * b + C1)
    np.testing.assert_allclose(mp[0, 5:-5, 5:-5], ref, rtol=0, atol=1e-14)
    # at the border the zero padding adds variance, so SSIM drops below that
    assert (mp[0, 0, :] < ref - 1e-6).all()


def test_single_pixel_image_closed_form():
    # a 1x1 image: the window holds x at its centre (weight w0) and 120 zeros,
    # so mu = w0 x, sigma^2 = w0 (1 - w0) x^2, sigma_xy = w0 (1 - w0) x y
    g1 = np.exp(-((np.arange(11) - 5.0) ** 2) / (2 * 1.5 ** 2))
    w0 = 1.0 / g1.sum() ** 2
    for x, y in [(0.2, 0.9), (0.8, 0.8), (1.0, 0.0), (0.5, 0.25)]:
        mean, _, g = oracle.ssim(np.full((1, 1, 1), x), np.full((1, 1, 1), y))
        v = w0 * (1 - w0)
        ref = (2 * w0 * w0 * x * y + C1) * (2 * v * x * y + C2) / ((w0 * w0 * (x * x + y * y) + C1) * (v * (x * x + y * y) + C2))
        assert abs(mean - ref) < 1e-13, (x, y)
        h = 1e-6
        fd = (oracle.ssim(np.full((1, 1, 1), x + h), np.full((1, 1, 1), y), False)[0] -
              oracle.ssim(np.full((1, 1, 1), x - h), np.full((1, 1, 1), y), False)[0]) / (2 * h)
        assert abs(g[0, 0, 0] - fd) < 1e-7 * max(1.0, abs(fd)), (x, y)


def test_map_matches_library_gaussian_filter():
    # local statistics from scipy's correlate with scipy's Gaussian window
    # (constant-zero boundary), variances via E[x^2] - mu^2
    X, Y = pair(1, (3, 27, 33))
    g1 = windows.gaussian(11, std=1.5)
    w2 = np.outer(g1, g1)
    w2 /= w2.sum()
    mean, mp, _ = oracle.ssim(X, Y, want_grad=False)
    ref = np.empty_like(X)
    for c in range(3):
        f = lambda a: ndimage.correlate(a, w2, mode="constant", cval=0.0)
        mx, my = f(X[c]), f(Y[c])
        vx, vy, cxy = f(X[c] * X[c]) - mx * mx, f(Y[c] * Y[c]) - my * my, f(X[c] * Y[c]) - mx * my
        ref[c] = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
    np.testing.assert_allclose(mp, ref, rtol=0, atol=1e-12)
    assert abs(mean - ref.mean()) < 1e-12


def test_symmetric_and_bounded():
    X, Y = pair(2)
    m1, mp1, _ = oracle.ssim(X, Y, False)
    m2, mp2, _ = oracle.ssim(Y, X, False)
    np.testing.assert_allclose(mp1, mp2, rtol=0, atol=1e-14)
    assert (np.abs(mp1) <= 1 + 1e-12).all() and m1 < 1


@pytest.mark.parametrize("shape", [(3, 9, 13), (1, 4, 17), (2, 12, 3)])
def test_gradient_matches_central_differences(shape):
    X, Y = pair(3, shape)
    _, _, g = oracle.ssim(X, Y)
    h = 1e-5
    fd = np.empty_like(X)
    for i in np.ndindex(X.shape):
        Xp = X.copy(); Xp[i] += h
        Xm = X.copy(); Xm[i] -= h
        fd[i] = (oracle.ssim(Xp, Y, False)[0] - oracle.ssim(Xm, Y, False)[0]) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 0
    np.testing.assert_allclose(g, fd, rtol=0, atol=1e-6 * scale)


def test_empty_image_counts_as_identical():
    mean, mp, g = oracle.ssim(np.zeros((3, 0, 5)), np.zeros((3, 0, 5)))
    assert mean == 1.0 and mp.size == 0 and g.size == 0
