"""Pins of the THI / THB oracle (Section IV, Section V-C)."""
import numpy as np
import pytest

import synth
from oracle import abcs, bounds


@pytest.fixture(scope="module")
def img():
    return synth.synth_image(41, 96, 80)


def _err(a, b):
    return float(np.sum((np.asarray(a, np.float64) - b) ** 2))


def test_full_subrate_recovers_exactly(img):
    for fn in (bounds.thi, bounds.thb):
        out = fn(img, 16, 1.0)
        rec = out[-1]
        assert np.max(np.abs(rec - img[:96, :80])) < 1e-9


@pytest.mark.parametrize("cr", [0.05, 0.1, 0.3])
def test_counts_and_error_energy(img, cr):
    coefs = bounds.coefficients(img, 16)
    m, keep, rec = bounds.thi(img, 16, cr)
    M, nB = bounds.total_measurements(img, 16, cr)
    assert m.sum() == M and m.max() <= 256
    dropped = float(np.sum(coefs[~keep] ** 2))
    assert abs(_err(rec, img) - dropped) <= 1e-6 * max(1.0, dropped)
    keep_b, rec_b = bounds.thb(img, 16, cr)
    assert np.all(keep_b.sum(axis=1) == M // nB)
    dropped_b = float(np.sum(coefs[~keep_b] ** 2))
    assert abs(_err(rec_b, img) - dropped_b) <= 1e-6 * max(1.0, dropped_b)
    # Parseval optimality: THI <= THB <= L-DCT-ZZ (same count per block as THB)
    k = abcs.budget(img, 16, cr, abcs.ZZ)[0]
    assert np.all(k == M // nB)
    rec_zz = abcs.reconstruct(abcs.sense(img, 16, k), 16, k, *img.shape)
    assert _err(rec, img) <= _err(rec_b, img) + 1e-6 <= _err(rec_zz, img) + 2e-6


def test_selection_matches_brute_force_sort():
    tiny = synth.synth_image(42, 32, 32)
    coefs = bounds.coefficients(tiny, 16)
    cands = sorted((-abs(coefs[b, z]), b, z) for b in range(coefs.shape[0]) for z in range(256))
    M, _ = bounds.total_measurements(tiny, 16, 0.2)
    want = np.zeros(coefs.shape, dtype=bool)
    for _, b, z in cands[:M]:
        want[b, z] = True
    _, keep, _ = bounds.thi(tiny, 16, 0.2)
    assert np.array_equal(keep, want)


def test_ties_go_to_lower_index():
    flat = np.full((32, 32), 100, np.uint8)     # every block: DC only, all equal
    m, keep, _ = bounds.thi(flat, 16, 2 / 1024 + 1e-9)   # M = 2 of 4 equal DC terms
    assert list(m) == [1, 1, 0, 0] and keep[0, 0] and keep[1, 0]


def test_pearson_special_cases():
    a = np.arange(10.0)
    assert bounds.pearson(a, 3 * a + 2) == pytest.approx(1.0)
    assert bounds.pearson(a, -a) == pytest.approx(-1.0)
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(50), rng.standard_normal(50)
    assert bounds.pearson(x, y) == pytest.approx(float(np.corrcoef(x, y)[0, 1]), abs=1e-12)


def test_pearson_p_closed_forms_and_library():
    # n = 3: t has 1 degree of freedom (Cauchy): p = 1 - (2/pi) atan|t|
    # n = 4: 2 degrees of freedom: p = 1 - |t| / sqrt(2 + t^2)
    for rho in (0.1, 0.5, -0.7, 0.95):
        t1 = abs(rho) * np.sqrt(1.0 / (1 - rho * rho))
        assert bounds.pearson_p(rho, 3) == pytest.approx(1 - 2 / np.pi * np.arctan(t1), rel=1e-12)
        t2 = abs(rho) * np.sqrt(2.0 / (1 - rho * rho))
        assert bounds.pearson_p(rho, 4) == pytest.approx(1 - t2 / np.sqrt(2 + t2 * t2), rel=1e-12)
    from scipy.stats import pearsonr
    rng = np.random.default_rng(3)
    for n in (10, 57, 400):
        x = rng.standard_normal(n)
        y = 0.3 * x + rng.standard_normal(n)
        r, p = pearsonr(x, y)
        assert bounds.pearson(x, y) == pytest.approx(r, abs=1e-12)
        assert bounds.pearson_p(bounds.pearson(x, y), n) == pytest.approx(p, rel=1e-9)
    assert bounds.pearson_p(1.0, 10) == 0.0 and np.isnan(bounds.pearson_p(float("nan"), 10))
