"""Pins of the oracle's budget scalars, BBV/DD statistics and apportionment
(Section V, Algorithms 1-2, eqs 16-23, Table 1)."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import abcs


def test_scalars_256_cr025():
    # 256x256, B = 16, C_R = 0.25: N = 65536, M = 16384, C_F = 4 (so L = 4,
    # X0 = 2, n_S = 4 by eqs 16-18), m1 = floor(256 / 8) = 32 (Alg 2 step 2).
    s = abcs.budget_scalars(256, 256, 16, 0.25, abcs.BBV)
    assert (s["N"], s["M"], s["CF"], s["L"], s["X0"], s["nS"]) == (65536, 16384, 4.0, 4, 2, 4)
    # eq 21 literally: 2 n_S n_B + (H + W) / L = 2*4*256 + 512/4
    assert s["M_BBV"] == 2 * 4 * 256 + 512 // 4 == 2176
    assert s["pool"] == 16384 - 2176 and s["cap"] == 256 - 8
    d = abcs.budget_scalars(256, 256, 16, 0.25, abcs.DD)
    assert (d["m1"], d["T"], d["pool"], d["cap"]) == (32, 60, 16384 - 256 * 32, 256 - 32)


@pytest.mark.parametrize("cr", [0.25, 0.4, 0.5])
def test_mbbv_equals_eq21_when_L_divides_B(cr):
    s = abcs.budget_scalars(512, 512, 16, cr, abcs.BBV)
    assert 16 % s["L"] == 0
    assert s["M_BBV"] == 2 * s["nS"] * s["nB"] + (512 + 512) // s["L"]


def test_table1_thresholds():
    # H = 256 column: C_F <= 2 -> 15, 2 < C_F < 3.33 -> 30, C_F >= 3.33 -> 60
    assert [abcs.dd_threshold(256, cf) for cf in (1.0, 2.0, 2.01, 3.3, 3.33, 4.0)] == [15, 15, 30, 30, 60, 60]
    # H = 512 column: 15 / 30 below 10 / 60 from 10 up
    assert [abcs.dd_threshold(512, cf) for cf in (2.0, 2.5, 9.99, 10.0, 20.0)] == [15, 30, 30, 60, 60]
    # 512x512 at C_R = 0.1 has C_F = 262144 / 26214 > 10
    assert abcs.budget_scalars(512, 512, 16, 0.1, abcs.DD)["T"] == 60
    assert abcs.budget_scalars(512, 512, 16, 0.5, abcs.DD)["T"] == 15


def test_domain_errors():
    with pytest.raises(abcs.DomainError):
        abcs.budget_scalars(256, 256, 16, 0.6, abcs.BBV)      # L = 1
    with pytest.raises(abcs.DomainError):
        abcs.budget_scalars(256, 256, 16, 0.0, abcs.ZZ)
    with pytest.raises(abcs.DomainError):
        abcs.budget_scalars(8, 8, 16, 0.5, abcs.ZZ)           # no whole block


def test_bbv_reverts_to_zz_when_ns_zero():
    # C_F > B gives n_S = 0 (eqs 16, 18): the budget is L-DCT-ZZ's
    img = synth.synth_image(5, 128, 128)
    s = abcs.budget_scalars(128, 128, 8, 0.1, abcs.BBV)
    assert s["nS"] == 0 and s["mode"] == abcs.ZZ
    k_bbv, _ = abcs.budget(img, 8, 0.1, abcs.BBV)
    k_zz, _ = abcs.budget(img, 8, 0.1, abcs.ZZ)
    assert np.array_equal(k_bbv, k_zz) and np.all(k_zz == math.floor(64 * 0.1))


def test_bbv_linear_ramp_closed_form():
    # I = a c + b r: every horizontal difference is a, every vertical one b,
    # so BBV_i = 2 n_S (|a| + |b|) for every block, edge blocks included.
    B, a, b = 8, 2, 3
    r, c = np.mgrid[0:32, 0:32]
    img = (a * c + b * r).astype(np.uint8)
    for L in (2, 3, 4):
        nS = B // L
        w = abcs.bbv_stat(img, B, L, L // 2, nS)
        assert np.all(w == 2 * nS * (a + b))


def test_bbv_hand_example():
    # 16x16 image of 2x2 blocks, B = 8, L = 4 -> X0 = 2, n_S = 2, sample
    # pairs at in-block offsets (1,2) and (5,6).  A step of height 50 between
    # columns 9 and 10 (inside block column 1, pair (1,2) of that block):
    #   top rows of blocks 1 and 3 each see |50| once,
    #   block 1's bottom term is block 3's top row (50),
    #   block 3 is in the last block row, so its bottom term is its own
    #   bottom row, which also crosses the step (50).
    img = np.zeros((16, 16), dtype=np.uint8)
    img[:, 10:] = 50
    w = abcs.bbv_stat(img, 8, 4, 2, 2)
    assert list(w) == [0, 100, 0, 100]
    # a horizontal step between rows 5 and 6 (block row 0, pair (5,6)) is seen
    # by the left-column samples of blocks 0 and 1; block 0's right term is
    # block 1's left column (50); block 1 is in the last block column and
    # uses its own right column (50).
    img = np.zeros((16, 16), dtype=np.uint8)
    img[6:, :] = 50
    assert list(abcs.bbv_stat(img, 8, 4, 2, 2)) == [100, 100, 0, 0]
    # a step exactly on the block border is never sampled
    img = np.zeros((16, 16), dtype=np.uint8)
    img[:, 8:] = 200
    assert list(abcs.bbv_stat(img, 8, 4, 2, 2)) == [0, 0, 0, 0]


def test_dd_stat_counts_dc_and_is_strict():
    # flat block of value 60/16*... : DC = sum / B.  B = 16, T = 60: a block
    # summing to exactly 960 has DC == T, which is not counted (strict >).
    B = 16
    img = np.zeros((16, 32), dtype=np.uint8)
    img[:, :16] = 0
    img[:15, :16] = 4          # sum 15*16*4 = 960 -> DC = 60 exactly
    img[:, 16:] = 4            # sum 1024 -> DC = 64 > 60
    n = abcs.dd_stat(img, B, 1, 60)
    assert list(n) == [0, 1]


def _brute_hamilton(P, w):
    """Among all integer allocations with sum P, the ones minimising the
    squared deviation from the exact quotas P w_i / S; of those the
    lexicographically greatest (ties to lower indices)."""
    n = len(w)
    S = sum(w)
    if S == 0:
        w, S = [1] * n, n
    quota = [Fraction(P * wi, S) for wi in w]
    best, best_val = None, None
    for a in itertools.product(range(P + 1), repeat=n):
        if sum(a) != P:
            continue
        val = sum((ai - qi) ** 2 for ai, qi in zip(a, quota))
        if best_val is None or val < best_val or (val == best_val and a > best):
            best, best_val = a, val
    return list(best)


@pytest.mark.parametrize("seed", range(40))
def test_apportion_uncapped_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 5))
    P = int(rng.integers(0, 9))
    w = [int(x) for x in rng.integers(0, 6, size=n)]
    if seed % 7 == 0:
        w = [0] * n
    if seed % 5 == 0 and n > 1:
        w[-1] = w[0]                      # force remainder ties
    a = abcs.apportion(P, w, cap=P + 1)
    assert list(a) == _brute_hamilton(P, w)


@pytest.mark.parametrize("seed", range(60))
def test_apportion_capped_invariants(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 40))
    cap = int(rng.integers(1, 20))
    P = int(rng.integers(0, cap * n + 1))
    w = rng.integers(0, 50, size=n)
    w[rng.random(n) < 0.3] = 0
    if seed % 4 == 0:
        w[rng.integers(0, n)] = 10000     # one dominant block overflows its cap
    a = abcs.apportion(P, w, cap)
    assert a.sum() == P and a.min() >= 0 and a.max() <= cap
    # monotone in the weight: a heavier block never gets fewer coefficients
    # than a lighter one, except by the single +1 of the remainder rule
    order = np.argsort(w, kind="stable")
    for i, j in zip(order[:-1], order[1:]):
        if w[j] > w[i]:
            assert a[j] >= a[i] - 1
    # blocks not at the cap got the Hamilton split of what the capped ones left
    free = np.nonzero(a < cap)[0]
    if free.size and free.size <= 4 and (P - cap * (n - free.size)) <= 8:
        rest = P - cap * (n - free.size)
        assert list(a[free]) == _brute_hamilton(rest, [int(w[i]) for i in free])


def test_apportion_cap_redistribution_example():
    # pool 30, cap 10, weights 8:1:1 -> floor quotas 24, 3, 3: block 0 hits the
    # cap (10) and the remaining 20 are re-split 1:1 -> 10, 10.
    assert list(abcs.apportion(30, [8, 1, 1], 10)) == [10, 10, 10]
    # pool 12, cap 10, weights 8:1:1 -> quotas 9.6, 1.2, 1.2 (no cap hit):
    # floors 9, 1, 1 and the single leftover goes to the largest remainder.
    assert list(abcs.apportion(12, [8, 1, 1], 10)) == [10, 1, 1]
    # pool 13: floors 10 (= cap) -> block 0 fixed at 10, 3 left -> 2, 1 (tie to index 1)
    assert list(abcs.apportion(13, [8, 1, 1], 10)) == [10, 2, 1]


@pytest.mark.parametrize("method", [abcs.BBV, abcs.DD, abcs.ZZ])
@pytest.mark.parametrize("cr", [0.1, 0.25, 0.5])
def test_budget_sums(method, cr):
    img = synth.synth_image(11, 256, 200)          # ragged: 200 = 12*16 + 8
    s = abcs.budget_scalars(256, 200, 16, cr, method)
    k, stat = abcs.budget(img, 16, cr, method)
    assert k.size == s["nB"] == 16 * 12
    if s["mode"] == abcs.BBV:
        assert k.sum() == s["pool"] and k.max() <= s["cap"]
    elif s["mode"] == abcs.DD:
        assert k.sum() == s["M"] and k.min() >= s["m1"] and k.max() <= 256
        assert stat.max() <= s["m1"]
    else:
        assert np.all(k == s["kz"]) and k.sum() <= s["M"]
