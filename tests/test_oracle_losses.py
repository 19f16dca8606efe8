"""Pins of the image-loss and Adam oracle (CPU)."""
import math

import numpy as np
import pytest

from oracle import losses as L


def _imgs(seed, shape=(3, 19, 23)):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, size=shape)
    y = np.clip(x + rng.normal(0, 0.1, size=shape), 0, 1)
    return x, y


def test_window_normalised_and_separable():
    w = L.gaussian_window()
    assert abs(w.sum() - 1.0) < 1e-15
    k = np.arange(11) - 5
    g = np.exp(-k * k / 4.5)
    g /= g.sum()
    np.testing.assert_allclose(w, np.outer(g, g), rtol=0, atol=1e-17)
    np.testing.assert_allclose(w, w.T, rtol=0, atol=0)


def test_ssim_of_identical_images_is_one():
    x, _ = _imgs(0)
    s, _ = L.ssim_map(x, x)
    np.testing.assert_allclose(s, 1.0, rtol=0, atol=1e-12)
    loss, g = L.image_loss(x, x)
    assert abs(loss) < 1e-12
    # x = y is a maximum of SSIM and L1's sign(0) = 0: zero gradient
    np.testing.assert_allclose(g, 0.0, atol=1e-12)


def test_constant_images_closed_form():
    """Away from the border the statistics of constant images are exact:
    SSIM = (2ab + C1) / (a^2 + b^2 + C1) (variances and covariance vanish)."""
    a, b = 0.7, 0.4
    x = np.full((1, 30, 30), a)
    y = np.full((1, 30, 30), b)
    s, _ = L.ssim_map(x, y)
    ref = (2 * a * b + L.C1) / (a * a + b * b + L.C1)
    np.testing.assert_allclose(s[0, 5:25, 5:25], ref, rtol=1e-11)  # FP64 rounding of 121-term window sums


def test_statistics_against_scipy_correlation():
    """The window sums, re-derived with scipy's correlation (zero border)."""
    from scipy import ndimage
    x, y = _imgs(1)
    s, st = L.ssim_map(x, y)
    w = L.gaussian_window()
    mx = np.stack([ndimage.correlate(c, w, mode="constant", cval=0.0) for c in x])
    exy = np.stack([ndimage.correlate(c, w, mode="constant", cval=0.0) for c in x * y])
    np.testing.assert_allclose(st["mx"], mx, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(st["exy"], exy, rtol=1e-12, atol=1e-15)


def test_gradient_against_finite_differences():
    x, y = _imgs(2, shape=(2, 13, 17))
    x[0, 3, 4] = y[0, 3, 4] + 0.05  # keep every |x - y| away from the L1 kink
    _, g = L.image_loss(x, y)
    rng = np.random.default_rng(5)
    for _ in range(40):
        idx = tuple(int(rng.integers(n)) for n in x.shape)
        if abs(x[idx] - y[idx]) < 1e-4:
            continue
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (L.image_loss(xp, y, grad=False)[0] - L.image_loss(xm, y, grad=False)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(abs(fd), 1e-4), (idx, fd, g[idx])


def test_l1_only_and_dssim_only_weights():
    x, y = _imgs(3)
    l1, _ = L.image_loss(x, y, lam=0.0, grad=False)
    assert abs(l1 - np.abs(x - y).mean()) < 1e-15
    d, _ = L.image_loss(x, y, lam=1.0, grad=False)
    s, _ = L.ssim_map(x, y)
    assert abs(d - (1.0 - s.mean())) < 1e-15


def test_adam_first_step_is_signed_learning_rate():
    """At step 1 the bias-corrected moments are g and g^2: the update is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(4)
    p, g = rng.normal(size=50), rng.normal(size=50)
    p1, m1, v1 = L.adam_step(p, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_adam_constant_gradient_keeps_unit_steps():
    """With a constant gradient the bias-corrected moments are exactly g and g^2
    at every step: every step moves by lr |g| / (|g| + eps)."""
    p = np.array([0.5, -2.0])
    g = np.array([0.3, -4.0])
    m = v = np.zeros(2)
    for t in range(1, 20):
        p, m, v = L.adam_step(p, g, m, v, t, 0.01)
    np.testing.assert_allclose(p, np.array([0.5, -2.0]) - 19 * 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13)
