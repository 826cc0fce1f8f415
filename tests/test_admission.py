"""CPU checks of admission control: a request's sizes (abcs_image_totals,
host code) against the oracle's budget of the same image (the length of y is
the sum of the per-block counts), and the batching rule."""
import numpy as np
import pytest

import synth
from oracle import abcs as orc


@pytest.mark.parametrize("B", [8, 16, 32])
@pytest.mark.parametrize("method", ["zz", "bbv", "dd"])
def test_image_totals_match_the_oracle_budget(B, method):
    import paper_2001_09632_amd as g
    rng = np.random.default_rng(B * 7 + len(method))
    for t in range(4):
        h, w = int(rng.integers(B, 200)), int(rng.integers(B, 200))
        cr = float(rng.uniform(0.05, 0.5))
        img = synth.synth_image(4000 + t, h, w)
        try:
            k, _ = orc.budget(img, B, cr, orc.METHOD_NAMES[method])
        except orc.DomainError:
            with pytest.raises(g.AbcsError, match="EDOMAIN"):
                g.image_totals(dict(height=h, width=w, block=B, subrate=cr, method=method))
            continue
        blocks, meas, pixels = g.image_totals(dict(height=h, width=w, block=B, subrate=cr, method=method))
        Hc, Wc, _, _, nB = orc.geometry(h, w, B)
        assert (blocks, pixels) == (nB, Hc * Wc)
        assert meas == int(k.sum()), (h, w, cr)


def test_image_totals_rejects_what_a_plan_rejects():
    import paper_2001_09632_amd as g
    with pytest.raises(g.AbcsError, match="EUNSUPPORTED"):
        g.image_totals(dict(height=64, width=64, block=12, subrate=0.2, method="zz"))
    with pytest.raises(g.AbcsError, match="EDOMAIN"):
        g.image_totals(dict(height=64, width=64, block=16, subrate=0.6, method="bbv"))
    with pytest.raises(g.AbcsError, match="EDOMAIN"):
        g.image_totals(dict(height=8, width=64, block=16, subrate=0.2, method="zz"))


def test_batches_keep_arrival_order_and_the_budget():
    import paper_2001_09632_amd as g
    rng = np.random.default_rng(3)
    reqs = [dict(height=int(rng.choice([64, 128, 256])), width=int(rng.choice([64, 128, 256])),
                 block=int(rng.choice([8, 16, 32])), subrate=float(rng.uniform(0.05, 0.5)),
                 method=str(rng.choice(["zz", "dd"]))) for _ in range(200)]
    adm = g.Admission(1 << 20)
    costs = [adm.cost(r) for r in reqs]
    bt = adm.batches(reqs)
    assert [i for b in bt for i in b] == list(range(len(reqs)))
    for j, b in enumerate(bt):
        used = sum(costs[i] for i in b)
        assert used <= adm.budget
        if j + 1 < len(bt):   # closed only because the next request did not fit
            assert used + costs[bt[j + 1][0]] > adm.budget
    assert adm.first_batch(reqs) == bt[0]
    # without the decoded images a request costs less
    assert g.Admission(1 << 20, decode=False).cost(reqs[0]) < costs[0]


def test_request_larger_than_the_budget_is_refused():
    import paper_2001_09632_amd as g
    adm = g.Admission(1000)
    with pytest.raises(ValueError):
        adm.batches([dict(height=64, width=64, block=16, subrate=0.2, method="zz")])
    with pytest.raises(ValueError):
        g.Admission(0)
