"""The package's PSNR/SSIM agree with the oracle's definitions."""
import numpy as np

from oracle import metrics
from paper_2001_09632_amd import quality


def test_quality_matches_oracle_metrics():
    rng = np.random.default_rng(0)
    ref = rng.integers(0, 256, size=(40, 52)).astype(np.float64)
    x = ref + rng.normal(0, 12, size=ref.shape)
    assert abs(quality.psnr(x, ref) - metrics.psnr(x, ref)) < 1e-9
    assert abs(quality.ssim(x, ref) - metrics.ssim(x, ref)) < 1e-9
