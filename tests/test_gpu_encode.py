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


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3", "bf16", "fp16"])
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


def _fused_entries():
    """A plan the one-launch encoder takes: 16 x 16 DCT images of at most 1024
    blocks, every rule (ZZ, BBV with and without samples, DD), ragged sizes,
    images of one block row and of a single block."""
    sizes = [(512, 512), (64, 48), (170, 181), (16, 16), (96, 500), (250, 130), (48, 272)]
    imgs = [synth.synth_image(5200 + i, h, w) for i, (h, w) in enumerate(sizes)]
    px, d = pack_images(imgs, pitch_pad=12)
    ent = []
    for i in range(len(imgs)):
        for m, cr in (("dd", 0.1), ("bbv", 0.3), ("zz", 0.2), ("bbv", 0.05), ("dd", 0.5), ("bbv", 0.5)):
            ent.append(dict(d[i], block=16, subrate=cr, method=m))
    return px, ent


def test_one_launch_encoder_equals_separate_calls():
    import torch
    import paper_2001_09632_amd as g
    px, ent = _fused_entries()
    a = Run(px, ent).budget().sense().reconstruct().fetch()
    b = Run(px, ent)
    nbytes = g.encode_workspace_bytes(b.plan)
    assert nbytes > 0
    ws = torch.full((nbytes,), 0x55, dtype=torch.uint8, device=b.px.device)   # contents do not matter
    for rep in range(3):                       # the workspace is reused as is
        b.out.fill_(float("nan"))
        g.encode(b.plan, b.px, b.k, b.off, b.stat, b.y, b.out, workspace=ws)
        b.fetch()
        _same(a, b)
        assert int(ws[4:8].view(torch.int32).item()) == 0   # no tile gave up waiting


def test_one_launch_encoder_on_the_benchmark_batch():
    """The 640-encoding batch (64 x 512^2, BBV and DD at five subrates):
    the one-launch encoder against the separate calls, bit for bit."""
    import torch
    import paper_2001_09632_amd as g
    imgs = [synth.synth_image(s, 512, 512) for s in range(1000, 1064)]
    px, d = pack_images(imgs)
    ent = [dict(d[i], block=16, subrate=cr, method=m) for m in ("bbv", "dd") for cr in (0.1, 0.2, 0.3, 0.4, 0.5)
           for i in range(64)]
    a = Run(px, ent).budget().sense().reconstruct().fetch()
    b = Run(px, ent)
    ws = torch.empty(g.encode_workspace_bytes(b.plan), dtype=torch.uint8, device=b.px.device)
    g.encode(b.plan, b.px, b.k, b.off, b.stat, b.y, b.out, workspace=ws)
    _same(a, b.fetch())


def test_encoder_workspace_only_for_eligible_plans():
    import paper_2001_09632_amd as g
    px, ent = _entries()                      # B = 8 and 32 and Walsh images: not eligible
    run = Run(px, ent)
    assert g.encode_workspace_bytes(run.plan) == 0
    big = g.Plan([dict(height=1024, width=1024, block=16, subrate=0.2, method="dd", pixel_offset=0)], features=())
    assert g.encode_workspace_bytes(big) == 0  # 4096 blocks: beyond the one-launch apportionment
