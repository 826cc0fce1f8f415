"""Launch splits on the GPU: every split gives the same bits as split 0 for
every block size, transform and a compensated and a single-pass precision,
on a batch with ragged tiles (widths that are not multiples of 16 blocks);
the tuner's timing call returns a time per split and leaves the table as it
was."""
import numpy as np
import pytest

import synth
from gpu_util import pack_images, device

pytestmark = pytest.mark.gpu


def _batch(B, transform):
    imgs = [synth.synth_image(1500 + i, h, w) for i, (h, w) in enumerate([(256, 336), (128, 120), (96, 520)])]
    px, d = pack_images(imgs)
    ents = [dict(d[i], block=B, subrate=cr, method=m, transform=transform)
            for i, (cr, m) in enumerate([(0.3, "dd"), (0.2, "bbv"), (0.45, "zz")])]
    return px, ents


def _run(g, plan, pxd, precision):
    import torch
    dev = device()
    k = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    off = torch.empty(plan.blocks, dtype=torch.int64, device=dev)
    st = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    y = torch.full((plan.meas,), float("nan"), dtype=torch.float32, device=dev)
    out = torch.full((plan.pixels,), float("nan"), dtype=torch.float32, device=dev)
    y2 = torch.full_like(y, float("nan"))
    out2 = torch.full_like(out, float("nan"))
    g.budget(plan, pxd, k, off, st)
    g.sense_decode(plan, pxd, k, off, y, out, precision=precision)
    g.sense(plan, pxd, k, off, y2, precision=precision)
    g.reconstruct(plan, y2, k, off, out2, precision=precision)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (y, out, y2, out2)]


@pytest.mark.parametrize("B", [8, 16, 32])
@pytest.mark.parametrize("transform", ["dct", "wht"])
def test_splits_give_the_same_bits(B, transform):
    import torch
    import paper_2001_09632_amd as g
    px, ents = _batch(B, transform)
    plan = g.Plan(ents, features=())
    pxd = torch.from_numpy(px).to(device())
    sc = g.plan_size_class(plan, B, transform)
    assert sc == 0
    precs = ["fp32"] if transform == "wht" else ["fp32", "bf16x3", "bf16"]
    try:
        for prec in precs:
            g.set_launch_table([])
            ref = _run(g, plan, pxd, prec)
            assert all(np.isfinite(a).all() for a in ref)
            for split in (1, 2):
                g.set_launch_table([dict(block=B, transform=transform, precision=prec, size_class=sc, split=split)])
                assert g.launch_split(B, transform, prec, sc) == split
                got = _run(g, plan, pxd, prec)
                for a, b in zip(ref, got):
                    assert np.array_equal(a, b), (B, transform, prec, split)
    finally:
        g.set_launch_table([])


def test_time_splits_times_each_split_and_keeps_the_table():
    import torch
    import paper_2001_09632_amd as g
    px, ents = _batch(16, "dct")
    plan = g.Plan(ents, features=())
    dev = device()
    pxd = torch.from_numpy(px).to(dev)
    k = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    off = torch.empty(plan.blocks, dtype=torch.int64, device=dev)
    st = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    y = torch.empty(plan.meas, dtype=torch.float32, device=dev)
    out = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    g.budget(plan, pxd, k, off, st)
    g.set_launch_table([dict(block=16, transform="dct", precision="fp32", size_class=0, split=2)])
    try:
        ms = g.time_splits(plan, pxd, k, off, y, out, "fp32", reps=3)
        assert len(ms) == 3 and all(v > 0 for v in ms)
        assert g.launch_split(16, "dct", "fp32", 0) == 2
    finally:
        g.set_launch_table([])
