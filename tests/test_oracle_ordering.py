"""Section VII-A's ordering of the budget rules, on the oracle and the
synthetic stand-in images: the adaptive rules decode at or above L-DCT-ZZ
(eq 26's fixed zigzag budget) at subrates 0.1 - 0.5.

The synthetic generator clips its sum of blobs, polygons and texture to
[0, 255], so some images hold perfectly flat (saturated) 16 x 16 blocks.
Such a block has no (or almost no) border variation, so AL-DCT-BBV gives it
no share of the pool and no coefficient at all (its phase-1 samples are
differences, not DCT coefficients), and the real-time decoder returns 0
there: those images are kept apart here.  AL-DCT-DD always measures the
first m1 coefficients of every block, DC included, so it keeps the ordering
on every image."""
import numpy as np
import pytest

import synth
from oracle import abcs as orc
from oracle import metrics

SEEDS = list(range(1000, 1012))
CRS = (0.1, 0.2, 0.3, 0.4, 0.5)


@pytest.fixture(scope="module")
def table():
    out = {}
    for s in SEEDS:
        img = synth.synth_image(s, 256, 256)
        for m in (orc.ZZ, orc.BBV, orc.DD):
            for cr in CRS:
                k, stat, y = orc.encode(img, 16, cr, m)
                rec = orc.reconstruct(y, 16, k, 256, 256)
                out[(s, m, cr)] = (metrics.psnr(rec, img.astype(np.float64)), k, stat)
    return out


def _empty(table, s, m, cr):
    return int((table[(s, m, cr)][1] == 0).sum())


def test_blocks_without_coefficients(table):
    """Only AL-DCT-BBV leaves blocks empty, and only blocks whose floor share
    of the pool is 0: P w_i < S (P the pool, S the sum of the weights; the
    capping rounds only raise P/S), i.e. a border variation far below the
    image's mean, as in saturated areas."""
    n_empty = 0
    for s in SEEDS:
        img = synth.synth_image(s, 256, 256)
        for cr in CRS:
            assert _empty(table, s, orc.ZZ, cr) == 0 and _empty(table, s, orc.DD, cr) == 0
            _, k, stat = table[(s, orc.BBV, cr)]
            pool = orc.budget_scalars(256, 256, 16, cr, orc.BBV)["pool"]
            w = stat.astype(np.int64)
            assert np.all(pool * w[k == 0] < w.sum()), (s, cr)
            n_empty += int((k == 0).sum())
    assert n_empty > 0      # the stand-in images do contain such blocks


def test_adaptive_rules_at_or_above_zigzag(table):
    """On the images where BBV leaves no block empty: DD above L-DCT-ZZ at
    every subrate; BBV at or above it at 0.2 - 0.5 and on the 0.1 - 0.5
    average (the Table 3 rows), and within 1 dB at 0.1, where one border
    sample per side (n_S = 1 at B = 16) carries the statistic (the paper's
    own margin there is 0.26 dB at 256^2, and its order reverses at 0.04).
    DD stays above L-DCT-ZZ on every image."""
    clean = [s for s in SEEDS if all(_empty(table, s, orc.BBV, cr) == 0 for cr in CRS)]
    assert len(clean) >= 6
    p = {m: {cr: np.mean([table[(s, m, cr)][0] for s in clean]) for cr in CRS} for m in (orc.ZZ, orc.BBV, orc.DD)}
    for cr in CRS:
        assert p[orc.DD][cr] > p[orc.ZZ][cr] + 0.5, (cr, p[orc.DD][cr], p[orc.ZZ][cr])
        assert p[orc.BBV][cr] >= p[orc.ZZ][cr] - (1.0 if cr == 0.1 else 0.0), (cr, p[orc.BBV][cr], p[orc.ZZ][cr])
    assert np.mean(list(p[orc.BBV].values())) > np.mean(list(p[orc.ZZ].values()))
    for cr in CRS:
        zz = np.mean([table[(s, orc.ZZ, cr)][0] for s in SEEDS])
        dd = np.mean([table[(s, orc.DD, cr)][0] for s in SEEDS])
        assert dd > zz, (cr, dd, zz)
