"""GPU parity of budget / sense / reconstruct against the FP64 oracle.

Bars: per-block budgets k, statistics (BBV_i, n_i) and offsets bit-exact;
measurements y within 1e-2 absolute (float32 transform of [0, 255] pixels:
with B = 16 every coefficient is a sum of 256 products whose magnitudes add
up to at most 255 * 4 * 4, and two 16-term float32 accumulations keep the
error below (2*16 + 2) * 2^-24 * 4080 < 1e-2); decoded pixels within 1e-3
absolute both of the oracle's decoding of the same measurements and, end to
end, of the oracle's decoding of its own float64 measurements (the inverse
transform is orthonormal, so the pixels' error has the same energy as the
measurements', which in practice stay near 1e-4).
"""
import numpy as np
import pytest

import synth
from oracle import abcs as orc

from gpu_util import Run, pack_images

pytestmark = pytest.mark.gpu

Y_TOL = 1e-2
PX_TOL = 1e-3


def _check_image(run, i, img, block, cr, method, check_y=True, check_px=True):
    got = run.image(i)
    k, stat = orc.budget(img, block, cr, method)
    assert np.array_equal(got["k"], k), f"k mismatch (image {i}, method {method}, C_R {cr})"
    assert np.array_equal(got["stat"], stat), f"stat mismatch (image {i})"
    assert np.array_equal(got["off"], orc.offsets(k)), f"offset mismatch (image {i})"
    assert got["y"].size == k.sum()
    if check_y or check_px:
        y = orc.sense(img, block, k)
    if check_y:
        err = np.max(np.abs(got["y"] - y)) if y.size else 0.0
        assert err < Y_TOL, f"y error {err} (image {i})"
    if check_px:
        H, W = img.shape
        rec = orc.reconstruct(got["y"].astype(np.float64), block, k, H, W)
        err = np.max(np.abs(got["out"] - rec))
        assert err < PX_TOL, f"pixel error {err} (image {i})"
        # end to end: the GPU's budget -> sense -> inverse transform against
        # the oracle's decoding of the oracle's own measurements
        rec = orc.reconstruct(y, block, k, H, W)
        err = np.max(np.abs(got["out"] - rec))
        assert err < PX_TOL, f"end-to-end pixel error {err} (image {i})"


def test_single_image_bbv_256():
    img = synth.synth_image(0, 256, 256)
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=16, subrate=0.25, method="bbv")]).budget().sense().reconstruct().fetch()
    _check_image(run, 0, img, 16, 0.25, orc.BBV)


def test_methods_subrates_ragged_sizes():
    imgs = [synth.synth_image(s, h, w) for s, (h, w) in enumerate([(256, 200), (64, 48), (170, 181), (16, 16)])]
    px, d = pack_images(imgs, pitch_pad=8)
    entries, cases = [], []
    for i, img in enumerate(imgs):
        for m in ("zz", "bbv", "dd"):
            for cr in (0.02, 0.1, 0.3, 0.5, 1.0):
                if m == "bbv" and cr > 0.5:
                    continue
                if img.shape == (16, 16) and m == "bbv" and cr < 0.1:
                    continue
                entries.append(dict(d[i], block=16, subrate=cr, method=m))
                cases.append((i, cr, orc.METHOD_NAMES[m]))
    run = Run(px, entries).budget().sense().reconstruct().fetch()
    for j, (i, cr, m) in enumerate(cases):
        _check_image(run, j, imgs[i], 16, cr, m)


def test_exact_recovery_full_subrate():
    img = synth.synth_image(77, 128, 96)
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=16, subrate=1.0, method=m) for m in ("zz", "dd")]).budget().sense() \
        .reconstruct().fetch()
    for j in range(2):
        got = run.image(j)
        assert np.all(got["k"] == 256)
        assert np.max(np.abs(got["out"] - img)) < PX_TOL


def test_degenerate_images():
    flat = np.full((64, 64), 128, np.uint8)                  # all weights 0 -> uniform split
    black = np.zeros((64, 64), np.uint8)
    one = np.full((64, 64), 90, np.uint8)
    one[16:32, 16:32] = synth.synth_image(3, 16, 16)          # one textured block: cap overflow
    one[16:32, 16:32:2] = 255
    checker = ((np.indices((48, 48)).sum(axis=0) % 2) * 255).astype(np.uint8)   # saturated texture
    dc_tie = np.zeros((32, 32), np.uint8)
    dc_tie[:15, :16] = 4                                      # block sum 960: DC == T = 60 exactly
    dc_tie[:, 16:] = 4
    imgs = [flat, black, one, checker, dc_tie]
    px, d = pack_images(imgs)
    entries, cases = [], []
    for i in range(len(imgs)):
        for m in ("bbv", "dd", "zz"):
            for cr in (0.1, 0.25, 0.5):
                entries.append(dict(d[i], block=16, subrate=cr, method=m))
                cases.append((i, cr, orc.METHOD_NAMES[m]))
    run = Run(px, entries).budget().sense().reconstruct().fetch()
    for j, (i, cr, m) in enumerate(cases):
        _check_image(run, j, imgs[i], 16, cr, m)


def _tie_blocks(seed, n):
    """n blocks whose coefficient C[8][0] is +-60 in exact arithmetic.

    Basis row 8 is s(x) / 4 with s = +1, -1, -1, +1, ... (cos of odd multiples
    of pi/4), so a block whose columns C of a random set of |R| columns hold a
    on rows with s = +1 and a - d elsewhere has C[8][0] = |R| d / 2.  With
    |R| d = 120 that is the DD threshold 60; the float64 value lands on, just
    above or just below 60 depending on the rounding of the basis."""
    s8 = np.sign(np.cos((2 * np.arange(16) + 1) * np.pi / 4))
    rng = np.random.default_rng(seed)
    out = []
    for t in range(n):
        R, d = [(8, 15), (10, 12), (12, 10), (15, 8), (4, 30), (6, 20), (5, 24)][t % 7]
        a = int(rng.integers(d, 256))
        cols = rng.choice(16, R, replace=False)
        blk = np.zeros((16, 16), np.uint8)
        blk[:, cols] = np.where(s8 > 0, a, a - d)[:, None]
        if rng.integers(0, 2):
            blk = np.roll(blk, 2, 0)                      # flips the sign of row 8
        out.append(blk)
    return out


def test_dd_many_exact_ties():
    """256 blocks, each with C[8][0] = +-T exactly in real arithmetic: every
    block sends coefficients into the float64 recheck, whose decisions (above,
    equal or below T by a few ulps in the canonical order) must be the
    oracle's."""
    blocks = _tie_blocks(11, 256)
    img = np.zeros((256, 256), np.uint8)
    for i, blk in enumerate(blocks):
        img[16 * (i // 16):16 * (i // 16) + 16, 16 * (i % 16):16 * (i % 16) + 16] = blk
    D = orc.dct_matrix(16)
    c80 = np.abs(orc.block_dct(np.stack(blocks).astype(np.float64), D)[:, 8, 0])
    assert np.all(np.abs(c80 - 60) < 1e-9) and (c80 > 60).any() and (c80 <= 60).any()
    crs = (0.29, 0.295)
    for cr in crs:
        assert orc.dd_threshold(256, 1 / cr) == 60
        assert orc.budget_scalars(256, 256, 16, cr, orc.DD)["m1"] >= 37     # (8, 0) has zigzag rank 36
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=16, subrate=cr, method="dd") for cr in crs]).budget().sense() \
        .reconstruct().fetch()
    for j, cr in enumerate(crs):
        _check_image(run, j, img, 16, cr, orc.DD)


def test_decoder_on_oracle_measurements():
    img = synth.synth_image(5, 256, 256)
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=16, subrate=0.2, method="dd")]).budget().fetch()
    k, _, y = orc.encode(img, 16, 0.2, orc.DD)
    import torch
    run.reconstruct(torch.from_numpy(y.astype(np.float32)).to(run.y.device)).fetch()
    rec = orc.reconstruct(y.astype(np.float32).astype(np.float64), 16, k, 256, 256)
    assert np.max(np.abs(run.image(0)["out"] - rec)) < PX_TOL


def test_runs_are_bitwise_repeatable():
    imgs = [synth.synth_image(s, 128, 128) for s in range(3)]
    px, d = pack_images(imgs)
    entries = [dict(d[i], block=16, subrate=0.3, method=m) for i in range(3) for m in ("bbv", "dd")]
    a = Run(px, entries).budget().sense().reconstruct().fetch()
    b = Run(px, entries).budget().sense().reconstruct().fetch()
    assert np.array_equal(a.h_k, b.h_k) and np.array_equal(a.h_y, b.h_y) and np.array_equal(a.h_out, b.h_out)


def test_batch_64x512_all_estimators_and_subrates():
    """The 64 x 512^2 batch with BBV and DD at C_R 0.1..0.5 in one plan, run
    exactly as the benchmark launches it (abcs_encode: budget, then sensing
    and the decoder in one pass): every budget, statistic and offset
    bit-exact; y and pixels compared in full on 8 images per combination."""
    seeds = list(range(1000, 1064))
    imgs = [synth.synth_image(s, 512, 512) for s in seeds]
    px, d = pack_images(imgs)
    entries, cases = [], []
    for m in ("bbv", "dd"):
        for cr in (0.1, 0.2, 0.3, 0.4, 0.5):
            for i in range(64):
                entries.append(dict(d[i], block=16, subrate=cr, method=m))
                cases.append((i, cr, orc.METHOD_NAMES[m]))
    run = Run(px, entries).encode().fetch()
    for j, (i, cr, m) in enumerate(cases):
        full = (i % 8 == 0)
        _check_image(run, j, imgs[i], 16, cr, m, check_y=full, check_px=full)
