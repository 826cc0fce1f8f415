"""PSNR and SSIM used to report reconstruction quality.

TEST INFRASTRUCTURE ONLY.

PSNR = 10 log10(255^2 / MSE) on the estimate clipped to [0, 255] against the
cropped ground truth (peak 255: 8-bit greyscale, Table 1 note).
SSIM follows Wang et al. (ref [18]): 11 x 11 Gaussian window with sigma 1.5,
K1 = 0.01, K2 = 0.03, L = 255, averaged over all windows that fit entirely in
the image.  The paper names the metrics but gives no parameters; these are the
defaults of the cited SSIM paper.

Parity: pinned by closed forms (constant images, constant offsets) in
tests/test_oracle_metrics.py.
"""

import math

import numpy as np


def psnr(x, ref):
    x = np.clip(np.asarray(x, dtype=np.float64), 0.0, 255.0)
    ref = np.asarray(ref, dtype=np.float64)[: x.shape[0], : x.shape[1]]
    mse = float(np.mean((x - ref) ** 2))
    return math.inf if mse == 0.0 else 10.0 * math.log10(255.0 ** 2 / mse)


def _gauss_window(size=11, sigma=1.5):
    ax = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(ax * ax) / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def _filter_valid(img, win):
    """Weighted sum over every window position that fits (explicit loops
    over the window taps)."""
    s = win.shape[0]
    H, W = img.shape
    out = np.zeros((H - s + 1, W - s + 1), dtype=np.float64)
    for a in range(s):
        for b in range(s):
            out = out + win[a, b] * img[a:a + H - s + 1, b:b + W - s + 1]
    return out


def ssim(x, ref, peak=255.0):
    x = np.clip(np.asarray(x, dtype=np.float64), 0.0, 255.0)
    y = np.asarray(ref, dtype=np.float64)[: x.shape[0], : x.shape[1]]
    win = _gauss_window()
    c1 = (0.01 * peak) ** 2
    c2 = (0.03 * peak) ** 2
    mx, my = _filter_valid(x, win), _filter_valid(y, win)
    sxx = _filter_valid(x * x, win) - mx * mx
    syy = _filter_valid(y * y, win) - my * my
    sxy = _filter_valid(x * y, win) - mx * my
    num = (2.0 * mx * my + c1) * (2.0 * sxy + c2)
    den = (mx * mx + my * my + c1) * (sxx + syy + c2)
    return float(np.mean(num / den))
