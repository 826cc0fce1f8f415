"""Property tests (hypothesis) on the oracle's apportionment and on the
library's host-side geometry and budget scalars, which must agree with the
oracle's for every descriptor (CPU only)."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import abcs as orc

SETTINGS = settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@st.composite
def apportion_case(draw):
    n = draw(st.integers(1, 40))
    w = draw(st.lists(st.integers(0, 10 ** 6), min_size=n, max_size=n))
    cap = draw(st.integers(0, 256))
    pool = draw(st.integers(0, cap * n))
    return np.array(w, dtype=np.int64), cap, pool


@SETTINGS
@given(apportion_case())
def test_apportion_sums_caps_and_orders(case):
    """Σk = pool, 0 <= k <= cap, and a heavier block never gets fewer
    coefficients than a lighter one (equal weights: the lower index first)."""
    w, cap, pool = case
    a = orc.apportion(pool, w, cap)
    assert int(a.sum()) == pool
    assert a.min() >= 0 and a.max() <= cap
    order = np.lexsort((np.arange(w.size), -w))   # by weight descending, then index
    assert np.all(np.diff(a[order]) <= 0)


@SETTINGS
@given(apportion_case())
def test_apportion_is_within_one_of_the_proportional_share(case):
    """Without caps in play every block's count is its exact share P w / S
    rounded down or up (Hamilton's method)."""
    w, cap, pool = case
    if w.sum() == 0:
        return
    big = int(pool) + 1          # no block can reach this cap
    a = orc.apportion(pool, w, big)
    share = pool * w / w.sum()
    assert np.all(a >= np.floor(share) - 1e-9) and np.all(a <= np.ceil(share) + 1e-9)


@st.composite
def descriptor(draw):
    B = draw(st.sampled_from([8, 16, 32]))
    h = draw(st.integers(1, 300))
    w = draw(st.integers(1, 300))
    cr = draw(st.floats(0.001, 1.0))
    m = draw(st.sampled_from(["zz", "bbv", "dd"]))
    return dict(height=h, width=w, block=B, subrate=cr, method=m)


@SETTINGS
@given(descriptor())
def test_library_geometry_and_sizes_match_the_oracle(d):
    """abcs_image_totals (the library's host-side derivation, the same code
    plan creation runs) against the oracle's budget scalars: blocks, pixels,
    and the coefficients in y (ZZ: n_B k_z; BBV: the pool; DD: M), and the
    same descriptors rejected."""
    import paper_2001_09632_amd as g
    method = {"zz": orc.ZZ, "bbv": orc.BBV, "dd": orc.DD}[d["method"]]
    try:
        s = orc.budget_scalars(d["height"], d["width"], d["block"], d["subrate"], method)
        if s["mode"] != orc.ZZ and s["pool"] > s["cap"] * s["nB"]:
            raise orc.DomainError("pool exceeds the blocks' capacity")
    except orc.DomainError:
        with pytest.raises(g.AbcsError, match="EDOMAIN"):
            g.image_totals(d)
        return
    blocks, meas, pixels = g.image_totals(d)
    assert blocks == s["nB"] and pixels == s["N"]
    want = {orc.ZZ: s["nB"] * s["kz"], orc.BBV: s.get("pool"), orc.DD: s["M"]}[s["mode"]]
    assert meas == want, (d, s)


@SETTINGS
@given(st.lists(descriptor(), min_size=1, max_size=30), st.integers(1 << 12, 1 << 22))
def test_admission_batches_cover_in_order_within_budget(descs, budget):
    import paper_2001_09632_amd as g
    adm = g.Admission(budget)
    ok, costs = [], []
    for d in descs:
        try:
            c = adm.cost(d)
        except g.AbcsError:
            continue
        if c <= budget:
            ok.append(d)
            costs.append(c)
    if not ok:
        return
    bt = adm.batches(ok)
    assert [i for b in bt for i in b] == list(range(len(ok)))
    for j, b in enumerate(bt):
        used = sum(costs[i] for i in b)
        assert used <= budget
        if j + 1 < len(bt):
            assert used + costs[bt[j + 1][0]] > budget
