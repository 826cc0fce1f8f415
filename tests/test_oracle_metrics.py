"""Closed-form pins of the quality metrics."""
import math

import numpy as np

from oracle import metrics


def test_psnr_constant_offset():
    ref = np.full((20, 20), 100.0)
    assert abs(metrics.psnr(ref + 5.0, ref) - 10 * math.log10(255.0 ** 2 / 25.0)) < 1e-12
    assert metrics.psnr(ref, ref) == math.inf
    # clipping to [0, 255] before the error is taken
    assert abs(metrics.psnr(np.full((4, 4), 300.0), np.full((4, 4), 250.0)) - 10 * math.log10(255.0 ** 2 / 25.0)) < 1e-12


def test_ssim_closed_forms():
    # identical images -> 1
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 255, size=(32, 40))
    assert abs(metrics.ssim(x, x) - 1.0) < 1e-12
    # constant images a, b: the variance terms are 0, so
    # SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 80.0, 120.0
    c1 = (0.01 * 255) ** 2
    got = metrics.ssim(np.full((16, 16), a), np.full((16, 16), b))
    assert abs(got - (2 * a * b + c1) / (a * a + b * b + c1)) < 1e-12
    # a constant offset leaves the structure term at 1: only luminance drops
    y = x + 10.0
    y = np.clip(y, 0, 255)
    assert 0.9 < metrics.ssim(np.clip(x, 0, 245), np.clip(x, 0, 245) + 10.0) < 1.0
