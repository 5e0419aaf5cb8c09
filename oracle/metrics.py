"""Image-quality metrics of Section 2.4.3 (MSE, PSNR, SSIM), FP64 (numpy).

Test infrastructure only.

The paper applies MSE, PSNR and SSIM to maximum-intensity projections against the
ground truth without stating their parameters.  Readings: images are the 60 dB display
values mapped to [0, 1] (data range L = 1); PSNR = 10 log10(L^2 / MSE); SSIM is the
index of Wang, Bovik, Sheikh and Simoncelli (IEEE TIP 2004) with an 11 x 11 Gaussian
window of standard deviation 1.5 (weights normalised to sum 1), K1 = 0.01, K2 = 0.03,
population (window-weighted) moments, averaged over the positions where the window lies
inside the image.
"""
from __future__ import annotations

import numpy as np

WIN = 11
SIGMA = 1.5
K1, K2 = 0.01, 0.03


def mse(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))


def psnr(a: np.ndarray, b: np.ndarray, data_range: float = 1.0) -> float:
    m = mse(a, b)
    return float('inf') if m == 0 else float(10.0 * np.log10(data_range ** 2 / m))


def gaussian_window(win: int = WIN, sigma: float = SIGMA) -> np.ndarray:
    """win x win weights w_i w_j, w_i proportional to exp(-i^2 / (2 sigma^2)), i centred, sum 1."""
    i = np.arange(win) - (win - 1) / 2.0
    w = np.exp(-i ** 2 / (2.0 * sigma ** 2))
    w2 = np.outer(w, w)
    return w2 / w2.sum()


def ssim_map(a: np.ndarray, b: np.ndarray, data_range: float = 1.0) -> np.ndarray:
    """SSIM at every position where the window fits: [ny - win + 1][nx - win + 1]."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    W = gaussian_window()
    n = W.shape[0]
    ny, nx = a.shape
    oy, ox = ny - n + 1, nx - n + 1
    if oy < 1 or ox < 1:
        raise ValueError('image smaller than the window')
    mu_a = np.zeros((oy, ox))
    mu_b = np.zeros((oy, ox))
    e_aa = np.zeros((oy, ox))
    e_bb = np.zeros((oy, ox))
    e_ab = np.zeros((oy, ox))
    for dy in range(n):          # weighted window sums, one window offset at a time
        for dx in range(n):
            w = W[dy, dx]
            pa = a[dy:dy + oy, dx:dx + ox]
            pb = b[dy:dy + oy, dx:dx + ox]
            mu_a += w * pa
            mu_b += w * pb
            e_aa += w * pa * pa
            e_bb += w * pb * pb
            e_ab += w * pa * pb
    va = e_aa - mu_a ** 2
    vb = e_bb - mu_b ** 2
    cab = e_ab - mu_a * mu_b
    c1 = (K1 * data_range) ** 2
    c2 = (K2 * data_range) ** 2
    return ((2 * mu_a * mu_b + c1) * (2 * cab + c2)) / ((mu_a ** 2 + mu_b ** 2 + c1) * (va + vb + c2))


def ssim(a: np.ndarray, b: np.ndarray, data_range: float = 1.0) -> float:
    return float(np.mean(ssim_map(a, b, data_range)))
