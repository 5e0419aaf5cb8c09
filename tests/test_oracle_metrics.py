"""Pins of the image-quality oracle (MSE, PSNR, SSIM)."""
import numpy as np
import pytest

from oracle import metrics


def test_mse_psnr_closed_forms():
    a = np.zeros((20, 30))
    b = np.full((20, 30), 0.1)
    assert abs(metrics.mse(a, b) - 0.01) < 1e-15
    assert abs(metrics.psnr(a, b) - 20.0) < 1e-12
    assert abs(metrics.psnr(a, b, data_range=10.0) - 40.0) < 1e-12
    assert metrics.psnr(a, a) == float('inf')


def test_window():
    W = metrics.gaussian_window()
    assert W.shape == (11, 11) and abs(W.sum() - 1) < 1e-15
    np.testing.assert_allclose(W, W.T, atol=0)
    # ratio of the centre weight to its neighbour is exp(1 / (2 * 1.5^2))
    assert abs(W[5, 5] / W[5, 6] - np.exp(1 / 4.5)) < 1e-12


def test_ssim_identity_and_symmetry():
    rng = np.random.default_rng(0)
    a = rng.random((32, 40))
    b = np.clip(a + 0.1 * rng.standard_normal(a.shape), 0, 1)
    assert abs(metrics.ssim(a, a) - 1.0) < 1e-12
    assert abs(metrics.ssim(a, b) - metrics.ssim(b, a)) < 1e-12
    assert metrics.ssim(a, b) < 1.0
    # more noise, lower similarity
    c = np.clip(a + 0.3 * rng.standard_normal(a.shape), 0, 1)
    assert metrics.ssim(a, c) < metrics.ssim(a, b)


def test_ssim_of_constant_images_is_the_luminance_term():
    """With no variance the contrast-structure factor is C2/C2 = 1, leaving
    (2 m1 m2 + C1) / (m1^2 + m2^2 + C1) at every position."""
    m1, m2 = 0.3, 0.7
    c1 = (0.01) ** 2
    want = (2 * m1 * m2 + c1) / (m1 ** 2 + m2 ** 2 + c1)
    got = metrics.ssim(np.full((15, 15), m1), np.full((15, 15), m2))
    assert abs(got - want) < 1e-12


def test_ssim_brute_force_on_a_tiny_image():
    """The shifted-window sums equal a plain per-position loop over the window pixels."""
    rng = np.random.default_rng(1)
    a = rng.random((12, 13))
    b = rng.random((12, 13))
    W = metrics.gaussian_window()
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    vals = []
    for y in range(12 - 10):
        for x in range(13 - 10):
            pa = a[y:y + 11, x:x + 11]
            pb = b[y:y + 11, x:x + 11]
            ma, mb = (W * pa).sum(), (W * pb).sum()
            va = (W * (pa - ma) ** 2).sum()
            vb = (W * (pb - mb) ** 2).sum()
            cab = (W * (pa - ma) * (pb - mb)).sum()
            vals.append((2 * ma * mb + c1) * (2 * cab + c2) / ((ma * ma + mb * mb + c1) * (va + vb + c2)))
    assert abs(metrics.ssim(a, b) - np.mean(vals)) < 1e-12


def test_ssim_rejects_images_smaller_than_the_window():
    with pytest.raises(ValueError):
        metrics.ssim(np.zeros((10, 30)), np.zeros((10, 30)))
