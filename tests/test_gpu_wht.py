"""GPU parity of Walsh-Hadamard sensing (Section IV's alternative transform)
against the FP64 oracle, for B = 8, 16 and 32 and in plans that mix it with
the DCT.

Bars as for the DCT: budgets, statistics and offsets bit-exact (DD on the
Walsh coefficients is evaluated in float64 in the definition's order); y
within 1e-2 (B = 8, 16) and 5e-2 (B = 32); decoded pixels within 1e-3 of the
oracle's decoding of the same measurements; IDA with the identity denoiser
within 2e-3 and sigma within 1e-5 relative.
"""
import numpy as np
import pytest

import synth
from oracle import abcs as orc
from oracle import ida as oida

from gpu_util import Run, pack_images, device

pytestmark = pytest.mark.gpu

PX_TOL = 1e-3
Y_TOL = {8: 1e-2, 16: 1e-2, 32: 5e-2}


def _check(run, j, img, B, cr, method, transform):
    got = run.image(j)
    k, stat = orc.budget(img, B, cr, method, transform)
    assert np.array_equal(got["k"], k), f"k mismatch (entry {j}, B {B}, {transform}, method {method}, C_R {cr})"
    assert np.array_equal(got["stat"], stat), f"stat mismatch (entry {j}, B {B}, {transform})"
    assert np.array_equal(got["off"], orc.offsets(k)), f"offsets (entry {j})"
    y = orc.sense(img, B, k, transform)
    if y.size:
        err = np.max(np.abs(got["y"] - y))
        assert err < Y_TOL[B], f"y error {err} (entry {j}, B {B}, {transform})"
    H, W = img.shape
    rec = orc.reconstruct(got["y"].astype(np.float64), B, k, H, W, transform)
    err = np.max(np.abs(got["out"] - rec))
    assert err < PX_TOL, f"pixel error {err} (entry {j}, B {B}, {transform})"


@pytest.mark.parametrize("B,sizes", [(8, [(72, 40), (131, 77)]), (16, [(64, 80), (256, 256), (200, 71)]),
                                     (32, [(96, 160), (64, 64)])])
def test_wht_methods_subrates(B, sizes):
    imgs = [synth.synth_image(1300 + 7 * i + B, h, w) for i, (h, w) in enumerate(sizes)]
    px, d = pack_images(imgs, pitch_pad=4)
    entries, cases = [], []
    for i, img in enumerate(imgs):
        for m in ("zz", "bbv", "dd"):
            for cr in (0.05, 0.1, 0.25, 0.5, 1.0):
                if m == "bbv" and cr > 0.5:
                    continue
                try:
                    orc.budget_scalars(img.shape[0], img.shape[1], B, cr, orc.METHOD_NAMES[m])
                except orc.DomainError:
                    continue
                entries.append(dict(d[i], block=B, subrate=cr, method=m, transform="wht"))
                cases.append((i, cr, orc.METHOD_NAMES[m]))
    run = Run(px, entries).budget().sense().reconstruct().fetch()
    for j, (i, cr, m) in enumerate(cases):
        _check(run, j, imgs[i], B, cr, m, "wht")


def test_dct_and_wht_in_one_plan():
    """The same pixels under both transforms and all three block sizes: the
    DCT B = 16 entries take the matrix-core kernels, the rest the vector-ALU
    ones."""
    imgs = [synth.synth_image(1400 + i, 128, 96) for i in range(2)]
    px, d = pack_images(imgs)
    entries, cases = [], []
    for i in range(2):
        for B in (8, 16, 32):
            for xf in ("dct", "wht"):
                for m in ("bbv", "dd"):
                    entries.append(dict(d[i], block=B, subrate=0.2, method=m, transform=xf))
                    cases.append((i, B, orc.METHOD_NAMES[m], xf))
    run = Run(px, entries).budget().sense().reconstruct().fetch()
    for j, (i, B, m, xf) in enumerate(cases):
        _check(run, j, imgs[i], B, 0.2, m, xf)


@pytest.mark.parametrize("B", [8, 16, 32])
def test_wht_ida_identity_matches_oracle(B):
    import torch
    import paper_2001_09632_amd as g
    imgs = [synth.synth_image(1500 + B, 96, 128), synth.synth_image(1501 + B, 64, 64)]
    px, d = pack_images(imgs)
    run = Run(px, [dict(d[0], block=B, subrate=0.25, method="dd", transform="wht"),
                   dict(d[1], block=B, subrate=0.2, method="zz", transform="wht")]).budget().sense().fetch()
    dev = device()
    iters = 6
    ws = torch.empty(g.ida_workspace_bytes(run.plan, "identity"), dtype=torch.uint8, device=dev)
    x = torch.full((run.plan.pixels,), float("nan"), dtype=torch.float32, device=dev)
    tr = torch.full((iters * run.plan.n,), float("nan"), dtype=torch.float32, device=dev)
    g.ida_refine(run.plan, run.y, run.k, run.off, x, iters, 2.0, "identity", sigma_trace=tr, workspace=ws)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    trh = tr.cpu().numpy().reshape(iters, run.plan.n)
    for i, img in enumerate(imgs):
        got = run.image(i)
        xo, sig = oida.ida(got["y"].astype(np.float64), got["k"], B, img.shape[0], img.shape[1], iters, 2.0,
                           transform="wht")
        di = run.plan.images[i]
        xi = xh[di["out_offset"]:di["out_offset"] + xo.size].reshape(xo.shape)
        assert np.allclose(trh[:, i], sig, rtol=1e-5, atol=0), f"sigma trace, image {i}"
        assert np.max(np.abs(xi - xo)) < 2e-3, f"x error, image {i}"


def test_wht_full_size_dd_512():
    """Four 512 x 512 images with B = 16, DD at two subrates: budgets exact
    at full size."""
    imgs = [synth.synth_image(1600 + i, 512, 512) for i in range(4)]
    px, d = pack_images(imgs)
    entries = [dict(d[i], block=16, subrate=cr, method="dd", transform="wht") for i in range(4) for cr in (0.1, 0.4)]
    run = Run(px, entries).budget().sense().reconstruct().fetch()
    for j, e in enumerate(entries):
        _check(run, j, imgs[j // 2], 16, e["subrate"], orc.DD, "wht")


def test_threshold_rejects_wht():
    import torch
    import paper_2001_09632_amd as g
    img = synth.synth_image(1700, 32, 32)
    px, d = pack_images([img])
    plan = g.Plan([dict(d[0], block=16, subrate=0.2, method="zz", transform="wht")])
    dev = device()
    pxd = torch.from_numpy(px).to(dev)
    m = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    ws = torch.empty(g.threshold_workspace_bytes(plan), dtype=torch.uint8, device=dev)
    with pytest.raises(g.AbcsError, match="EUNSUPPORTED"):
        g.threshold(plan, pxd, m, rule="thi", workspace=ws)
