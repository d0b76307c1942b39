"""Image similarity of a reslice against the acquired frame at the same pose (the paper's
quantitative evaluation: normalised cross-correlation and the structural similarity index between
resliced images and their ground truth, Sec. 3, "Quantitative image similarity").

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names the two measures and no variant of either; the readings here are the standard
ones, in FP64:
  NCC   zero-mean normalised cross-correlation over the pixels the reslice assigns (finite):
        sum (a - mean a)(b - mean b) / sqrt(sum (a - mean a)^2 sum (b - mean b)^2);
  SSIM  Wang et al.'s index with an 11 x 11 Gaussian window (sigma 1.5, normalised to sum 1),
        K1 = 0.01, K2 = 0.03 and dynamic range L = 255, averaged over the pixels whose whole
        window lies inside the image and is assigned in the reslice.
Unassigned (NaN) reslice pixels carry no value, so they are left out of both rather than filled.
"""
from __future__ import annotations

import math

import numpy as np

WINDOW = 11
SIGMA = 1.5
K1, K2, L = 0.01, 0.03, 255.0


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """size x size Gaussian weights exp(-(x^2 + y^2) / (2 sigma^2)) about the centre, summing to 1."""
    r = size // 2
    g = np.empty((size, size), np.float64)
    for y in range(size):
        for x in range(size):
            g[y, x] = math.exp(-((x - r) ** 2 + (y - r) ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def ncc(image, frame):
    """(NCC, number of pixels used): the reslice's finite pixels against the frame's."""
    a = np.asarray(image, np.float64)
    b = np.asarray(frame, np.float64)
    m = np.isfinite(a)
    n = int(m.sum())
    if n < 2:
        return float("nan"), n
    a, b = a[m], b[m]
    da, db = a - a.mean(), b - b.mean()
    den = math.sqrt(float((da * da).sum()) * float((db * db).sum()))
    return (float((da * db).sum()) / den if den > 0.0 else float("nan")), n


def ssim(image, frame):
    """(mean SSIM, number of windows used) over every pixel whose whole window is inside the
    image and finite in the reslice."""
    a = np.asarray(image, np.float64)
    b = np.asarray(frame, np.float64)
    g = gaussian_window()
    r = WINDOW // 2
    c1, c2 = (K1 * L) ** 2, (K2 * L) ** 2
    H, W = a.shape
    total, n = 0.0, 0
    for j in range(r, H - r):
        for i in range(r, W - r):
            wa = a[j - r:j + r + 1, i - r:i + r + 1]
            if not np.isfinite(wa).all():
                continue
            wb = b[j - r:j + r + 1, i - r:i + r + 1]
            ma, mb = float((g * wa).sum()), float((g * wb).sum())
            va = float((g * wa * wa).sum()) - ma * ma
            vb = float((g * wb * wb).sum()) - mb * mb
            cab = float((g * wa * wb).sum()) - ma * mb
            total += ((2.0 * ma * mb + c1) * (2.0 * cab + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2))
            n += 1
    return (total / n if n else float("nan")), n
