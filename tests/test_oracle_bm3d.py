"""Pins of the BM3D oracle (plain IDA denoiser, ref [22] of the paper)."""
import math

import numpy as np
import pytest

import synth
from oracle import bm3d, metrics


def test_sigma_zero_is_identity():
    v = np.random.default_rng(0).uniform(0, 255, size=(24, 32))
    assert np.array_equal(bm3d.bm3d(v, 0.0), v)


def test_constant_image_stays_constant():
    # every group holds identical flat patches: only the DC of the 3D spectrum
    # is non-zero.  Stage 1 keeps it (8 * 100 * sqrt(16) > 2.7 sigma), stage 2
    # (32-member groups) shrinks it by the Wiener factor B^2 / (B^2 + sigma^2),
    # B = 8 * 100 * sqrt(32).
    v = np.full((32, 40), 100.0)
    out = bm3d.bm3d(v, 20.0)
    assert np.ptp(out) < 1e-9
    b2 = 800.0 ** 2 * 32
    assert abs(out[0, 0] - 100.0 * b2 / (b2 + 400.0)) < 1e-9
    assert np.max(np.abs(bm3d.stage1(v, 20.0) - 100.0)) < 1e-9


def test_haar_closed_forms():
    assert np.allclose(bm3d.haar_fwd(np.array([1.0, 1.0])), [math.sqrt(2), 0.0])
    # [a, b, c, d] -> [(a+b+c+d)/2, (a+b-c-d)/2, (a-b)/sqrt2, (c-d)/sqrt2]
    h = bm3d.haar_fwd(np.array([1.0, 3.0, 6.0, 2.0]))
    assert np.allclose(h, [6.0, -2.0, -2.0 / math.sqrt(2), 4.0 / math.sqrt(2)])
    x = np.random.default_rng(1).normal(size=(16, 3))
    assert np.allclose(bm3d.haar_inv(bm3d.haar_fwd(x)), x)
    assert np.allclose((bm3d.haar_fwd(x) ** 2).sum(axis=0), (x ** 2).sum(axis=0))


def test_3d_transform_orthonormal_and_dc():
    D = bm3d.dct8()
    g = np.random.default_rng(2).uniform(0, 255, size=(8, 8, 8))
    s = bm3d.transform3d(g, D)
    assert np.allclose(bm3d.inverse3d(s, D), g)
    assert np.isclose((s ** 2).sum(), (g ** 2).sum())
    # DC of the 3D spectrum = sum / sqrt(64 n)
    assert np.isclose(s[0, 0, 0], g.sum() / math.sqrt(64 * 8))


def test_reference_positions_cover_the_image():
    assert bm3d.ref_positions(8) == [0]
    assert bm3d.ref_positions(17) == [0, 3, 6, 9]
    assert bm3d.ref_positions(20) == [0, 3, 6, 9, 12]


def test_grouping_finds_planted_copies():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(48, 48)).astype(np.float64)
    pat = rng.integers(0, 256, size=(8, 8)).astype(np.float64)
    for (y, x) in [(9, 12), (20, 3), (25, 28)]:
        img[y:y + 8, x:x + 8] = pat
    # reference at (9, 12), window rows 0..28, columns 0..31: copies at
    # distance 0; everything else is far
    # (random patches differ by ~2 * 255^2 / 12 per pixel >> tau).  Three
    # members cut to the largest power of two: the reference and the first
    # copy in raster order.
    assert bm3d.match(img, 9, 12, bm3d.TAU_HT, bm3d.N2_HT) == [(9, 12), (20, 3)]
    # with the planted copies at equal distance, raster order decides
    img2 = img.copy()
    img2[20:28, 3:11] = rng.integers(0, 256, size=(8, 8))
    assert bm3d.match(img2, 9, 12, bm3d.TAU_HT, bm3d.N2_HT) == [(9, 12), (25, 28)]
    # a copy outside the clipped window is not seen
    img3 = img2.copy()
    img3[25:33, 28:36] = rng.integers(0, 256, size=(8, 8))
    img3[30:38, 30:38] = pat
    assert bm3d.match(img3, 9, 12, bm3d.TAU_HT, bm3d.N2_HT) == [(9, 12)]


def test_kaiser_window_symmetric_peak_one_free():
    K = bm3d.kaiser2d()
    assert np.allclose(K, K.T) and np.allclose(K, K[::-1, ::-1])
    assert K.max() <= 1.0 + 1e-12 and K.min() > 0


@pytest.mark.parametrize("sigma", [15.0, 30.0])
def test_denoising_reduces_error(sigma):
    clean = synth.synth_image(7, 48, 56).astype(np.float64)
    noisy = clean + np.random.default_rng(4).normal(0, sigma, size=clean.shape)
    out = bm3d.bm3d(noisy, sigma)
    assert metrics.psnr(out, clean) > metrics.psnr(noisy, clean) + 3.0


def test_kaiser_window_closed_form():
    # w[i] = I0(beta sqrt(1 - t^2)) / I0(beta), t = 2i/(n-1) - 1 (Kaiser's
    # window; I0 from scipy), the 2-D window its outer product
    from scipy.special import i0
    t = 2.0 * np.arange(8) / 7.0 - 1.0
    w = i0(bm3d.KAISER_BETA * np.sqrt(1.0 - t * t)) / i0(bm3d.KAISER_BETA)
    assert np.allclose(bm3d.kaiser2d(), np.outer(w, w), rtol=1e-13, atol=0)
    assert w[0] == pytest.approx(1.0 / i0(2.0)) and w[0] == pytest.approx(0.4386, abs=1e-4)


def _single_member_image(seed):
    """An 8 x 11 image of uniform noise: two reference positions (columns 0
    and 3) whose groups hold only the reference (every other candidate
    patch is far beyond both thresholds)."""
    img = np.random.default_rng(seed).uniform(0, 255, size=(8, 11))
    win = [img[:, x:x + 8] for x in range(4)]
    for a in range(4):
        for b in range(a + 1, 4):
            assert np.sum((win[a] - win[b]) ** 2) / 64.0 > 2 * bm3d.TAU_HT
    assert bm3d.ref_positions(11) == [0, 3] and bm3d.ref_positions(8) == [0]
    return img


def _aggregate_two(estimates, weights):
    """Weighted Kaiser-window average of two 8 x 8 estimates at columns 0
    and 3 of an 8 x 11 image (Kaiser window from its closed form)."""
    from scipy.special import i0
    t = 2.0 * np.arange(8) / 7.0 - 1.0
    k = i0(2.0 * np.sqrt(1.0 - t * t)) / i0(2.0)
    K = np.outer(k, k)
    num, den = np.zeros((8, 11)), np.zeros((8, 11))
    for x, e, w in zip((0, 3), estimates, weights):
        num[:, x:x + 8] += w * K * e
        den[:, x:x + 8] += w * K
    return num / den


def test_stage1_group_weight_is_inverse_surviving_count():
    # groups of one patch: the 3-D transform is the patch's 2-D DCT (a
    # length-1 Haar transform is the identity), so stage 1 is hard
    # thresholding of each patch's DCT (scipy's orthonormal DCT here), and
    # where the two patches overlap the estimate is their Kaiser-weighted
    # average with weights 1 / (sigma^2 N_har)
    from scipy.fft import dctn, idctn
    sigma = 30.0
    img = _single_member_image(8)
    est, nhar = [], []
    for x in (0, 3):
        c = dctn(img[:, x:x + 8], norm="ortho")
        c[np.abs(c) <= 2.7 * sigma] = 0.0
        nhar.append(int(np.count_nonzero(c)))
        est.append(idctn(c, norm="ortho"))
    assert nhar[0] != nhar[1]
    want = _aggregate_two(est, [1.0 / (sigma * sigma * n) for n in nhar])
    got = bm3d.stage1(img, sigma)
    assert np.max(np.abs(got - want)) < 1e-9
    # the weights matter: equal weights give a visibly different image
    assert np.max(np.abs(_aggregate_two(est, [1.0, 1.0]) - want)) > 0.1


def test_stage2_group_weight_is_inverse_wiener_energy():
    # groups of one patch again (matched on the stage-1 estimate `basic`):
    # each patch's DCT is scaled by W = B^2 / (B^2 + sigma^2), B the DCT of
    # the same patch of `basic`, and the group weight is 1 / (sigma^2 ||W||^2)
    from scipy.fft import dctn, idctn
    sigma = 40.0
    basic = _single_member_image(9)
    noisy = basic + np.random.default_rng(10).normal(0, sigma, size=basic.shape)
    est, wts = [], []
    for x in (0, 3):
        b = dctn(basic[:, x:x + 8], norm="ortho")
        W = b * b / (b * b + sigma * sigma)
        est.append(idctn(W * dctn(noisy[:, x:x + 8], norm="ortho"), norm="ortho"))
        wts.append(1.0 / (sigma * sigma * np.sum(W * W)))
    assert abs(wts[0] / wts[1] - 1.0) > 0.05
    want = _aggregate_two(est, wts)
    got = bm3d.stage2(noisy, basic, sigma)
    assert np.max(np.abs(got - want)) < 1e-9
    assert np.max(np.abs(_aggregate_two(est, [1.0, 1.0]) - want)) > 0.01
