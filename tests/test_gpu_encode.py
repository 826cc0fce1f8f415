"""abcs_encode (budget, sensing and the decoder's image in one call) against
the three separate calls: budgets, statistics, offsets, measurements and
decoded pixels identical bit for bit, for every launch class (B = 8, 16,
32; DCT and Walsh-Hadamard), ragged sizes, every rule, and the 16-bit
precision modes.  The separate calls are checked against the oracle by
test_gpu_abcs.py and test_gpu_blocks.py; the 64 x 512^2 batch runs through
abcs_encode there as well."""
import numpy as np
import pytest

import synth

from gpu_util import Run, pack_images

pytestmark = pytest.mark.gpu


def _entries():
    sizes = [(256, 200), (64, 48), (170, 181), (96, 96), (48, 272)]
    imgs = [synth.synth_image(5000 + i, h, w) for i, (h, w) in enumerate(sizes)]
    px, d = pack_images(imgs, pitch_pad=4)
    ent = []
    for i in range(len(imgs)):
        for B in (8, 16, 32):
            for xf in ("dct", "wht"):
                for m, cr in (("zz", 0.2), ("bbv", 0.3), ("dd", 0.15), ("dd", 0.5)):
                    if min(sizes[i]) < B:
                        continue
                    ent.append(dict(d[i], block=B, subrate=cr, method=m, transform=xf))
    return px, ent


def _same(a, b):
    for name in ("h_k", "h_off", "h_stat", "h_y", "h_out"):
        x, y = getattr(a, name), getattr(b, name)
        assert x.shape == y.shape and np.array_equal(x, y, equal_nan=True), name


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16"])
def test_encode_equals_separate_calls(precision):
    px, ent = _entries()
    a = Run(px, ent)
    import paper_2001_09632_amd as g
    g.budget(a.plan, a.px, a.k, a.off, a.stat)
    g.sense(a.plan, a.px, a.k, a.off, a.y, precision=precision)
    g.reconstruct(a.plan, a.y, a.k, a.off, a.out, precision=precision)
    a.fetch()
    b = Run(px, ent).encode(precision=precision).fetch()
    _same(a, b)


def test_encode_without_decoder_output():
    px, ent = _entries()
    a = Run(px, ent).budget().sense().fetch()
    b = Run(px, ent).encode(out=False).fetch()
    _same(a, b)                       # out untouched (NaN) in both
    assert np.all(np.isnan(b.h_out))


def test_encode_rejects_bad_arguments_before_launching():
    import torch
    import paper_2001_09632_amd as g
    px, ent = _entries()
    run = Run(px, ent)
    with pytest.raises(g.AbcsError):
        g.encode(run.plan, run.px, run.k, run.off, run.stat, run.y, run.out[1:])   # misaligned output
    with pytest.raises(g.AbcsError):
        g.encode(run.plan, run.px[:16], run.k, run.off, run.stat, run.y, run.out)  # pixel buffer too small
    torch.cuda.synchronize()
    assert bool((run.k == -7).all()) and bool(torch.isnan(run.y).all())


def test_sense_decode_after_budget_equals_separate_calls():
    import paper_2001_09632_amd as g
    px, ent = _entries()
    a = Run(px, ent).budget().sense().reconstruct().fetch()
    b = Run(px, ent).budget()
    g.sense_decode(b.plan, b.px, b.k, b.off, b.y, b.out)
    _same(a, b.fetch())


def test_plan_without_optional_tables():
    """An encoder/decoder-only plan runs encode, reconstruct and the
    identity-denoiser IDA loop, and refuses the calls that need the
    denoisers' or the bounds' tables with EINVAL before launching."""
    import torch
    import paper_2001_09632_amd as g
    from gpu_util import device
    img = synth.synth_image(5100, 64, 96)
    px, d = pack_images([img])
    ent = [dict(d[0], block=16, subrate=0.25, method="dd")]
    full = Run(px, ent).encode().fetch()
    run = Run(px, ent)
    run.plan = g.Plan(ent, features=())
    run.encode().fetch()
    assert np.array_equal(run.h_out, full.h_out)
    dev = device()
    x = torch.zeros(run.plan.pixels, dtype=torch.float32, device=dev)
    ws = torch.empty(g.ida_workspace_bytes(run.plan, "bm3d"), dtype=torch.uint8, device=dev)
    g.ida_refine(run.plan, run.y, run.k, run.off, x, 2, 2.0, "identity", workspace=ws)
    with pytest.raises(g.AbcsError, match="ABCS_PLAN_DENOISE"):
        g.ida_refine(run.plan, run.y, run.k, run.off, x, 2, 2.0, "bm3d", workspace=ws)
    m = torch.zeros(run.plan.blocks, dtype=torch.int32, device=dev)
    tws = torch.empty(g.threshold_workspace_bytes(run.plan), dtype=torch.uint8, device=dev)
    with pytest.raises(g.AbcsError, match="ABCS_PLAN_BOUNDS"):
        g.threshold(run.plan, run.px, m, rule="thi", workspace=tws)
    torch.cuda.synchronize()
