"""Image-quality figures reported next to throughput (host numpy).

PSNR = 10 log10(255^2 / MSE) of the estimate clipped to [0, 255] against the
8-bit reference; SSIM (Wang et al., ref [18] of the paper) with an 11x11
Gaussian window of standard deviation 1.5, K1 = 0.01, K2 = 0.03, L = 255,
averaged over the window positions that fit inside the image.  Evaluation
support only: nothing on the sensing or reconstruction path uses it.
"""
import math

import numpy as np


def psnr(x, ref):
    x = np.clip(np.asarray(x, dtype=np.float64), 0.0, 255.0)
    r = np.asarray(ref, dtype=np.float64)
    mse = float(np.mean((x - r) ** 2))
    return math.inf if mse == 0.0 else 10.0 * math.log10(65025.0 / mse)


def _gauss1d(n=11, s=1.5):
    t = np.arange(n) - (n - 1) / 2.0
    g = np.exp(-t * t / (2 * s * s))
    return g / g.sum()


def _blur_valid(a, g):
    n = g.size
    rows = sum(g[i] * a[:, i:a.shape[1] - n + 1 + i] for i in range(n))
    return sum(g[i] * rows[i:rows.shape[0] - n + 1 + i, :] for i in range(n))


def ssim(x, ref):
    x = np.clip(np.asarray(x, dtype=np.float64), 0.0, 255.0)
    y = np.asarray(ref, dtype=np.float64)
    g = _gauss1d()
    c1, c2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    mx, my = _blur_valid(x, g), _blur_valid(y, g)
    vx = _blur_valid(x * x, g) - mx * mx
    vy = _blur_valid(y * y, g) - my * my
    cxy = _blur_valid(x * y, g) - mx * my
    m = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    return float(m.mean())
