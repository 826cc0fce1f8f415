"""GPU parity for block sizes 8 and 32 and for plans that mix B = 8, 16 and
32, against the FP64 oracle.  Sensing and the inverse transform run on the
matrix cores (B = 8: four blocks per 16x16 transform; B = 32: 2x2 tiles of
16x16), the DD statistics and the IDA step on the vector ALUs.

Bars as for B = 16: budgets, statistics and offsets bit-exact; decoded pixels
within 1e-3 of the oracle's decoding of the same measurements.  y: within
1e-2 (B = 8) and 5e-2 (B = 32) absolute: the coefficients grow with B (up to
255 B) and the float32 inputs of each product are rounded once.
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


def _check(run, j, img, B, cr, method):
    got = run.image(j)
    k, stat = orc.budget(img, B, cr, method)
    assert np.array_equal(got["k"], k), f"k mismatch (entry {j}, B {B}, method {method}, C_R {cr})"
    assert np.array_equal(got["stat"], stat), f"stat mismatch (entry {j}, B {B})"
    assert np.array_equal(got["off"], orc.offsets(k)), f"offsets (entry {j})"
    y = orc.sense(img, B, k)
    if y.size:
        err = np.max(np.abs(got["y"] - y))
        assert err < Y_TOL[B], f"y error {err} (entry {j}, B {B})"
    H, W = img.shape
    rec = orc.reconstruct(got["y"].astype(np.float64), B, k, H, W)
    err = np.max(np.abs(got["out"] - rec))
    assert err < PX_TOL, f"pixel error {err} (entry {j}, B {B})"


@pytest.mark.parametrize("B,sizes", [(8, [(72, 40), (256, 256), (8, 8), (131, 77)]),
                                     (32, [(96, 160), (256, 256), (32, 32), (200, 71)])])
def test_block_size_methods_subrates(B, sizes):
    imgs = [synth.synth_image(300 + 7 * i + B, h, w) for i, (h, w) in enumerate(sizes)]
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
                entries.append(dict(d[i], block=B, subrate=cr, method=m))
                cases.append((i, cr, orc.METHOD_NAMES[m]))
    run = Run(px, entries).budget().sense().reconstruct().fetch()
    for j, (i, cr, m) in enumerate(cases):
        _check(run, j, imgs[i], B, cr, m)


def test_mixed_block_sizes_in_one_plan():
    imgs = [synth.synth_image(400 + i, 128, 96) for i in range(3)]
    px, d = pack_images(imgs)
    entries, cases = [], []
    for i, B in enumerate((8, 16, 32)):
        for m in ("bbv", "dd"):
            for cr in (0.1, 0.3):
                entries.append(dict(d[i], block=B, subrate=cr, method=m))
                cases.append((i, B, cr, orc.METHOD_NAMES[m]))
    run = Run(px, entries).budget().sense().reconstruct().fetch()
    for j, (i, B, cr, m) in enumerate(cases):
        _check(run, j, imgs[i], B, cr, m)


@pytest.mark.parametrize("B", [8, 32])
def test_dd_dc_ties(B):
    """Blocks whose pixel sum is B T make DC = T exactly (DC = sum / B); with
    one pixel more DC = T + 1/B.  The counts must be the oracle's."""
    rng = np.random.default_rng(B)
    img = np.zeros((8 * B, 8 * B), np.uint8)
    for by in range(8):
        for bx in range(8):
            blk = np.zeros(B * B, np.int64)
            total = B * 60 + (1 if (by + bx) % 3 == 0 else 0)     # T = 60 below
            idx = rng.choice(B * B, size=total // 30 + 1, replace=False)
            blk[idx] = 30
            blk[idx[0]] += total - blk.sum()
            img[by * B:(by + 1) * B, bx * B:(bx + 1) * B] = blk.reshape(B, B).astype(np.uint8)
    H = img.shape[0]
    cr = 0.1 if H >= 512 else 0.25
    assert orc.dd_threshold(H, 1 / cr) == 60
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=B, subrate=cr, method="dd")]).budget().sense().reconstruct().fetch()
    _check(run, 0, img, B, cr, orc.DD)


@pytest.mark.parametrize("B", [8, 32])
def test_ida_identity_matches_oracle(B):
    import torch
    import paper_2001_09632_amd as g
    imgs = [synth.synth_image(500 + B, 96, 128), synth.synth_image(501 + B, 64, 64)]
    px, d = pack_images(imgs)
    run = Run(px, [dict(d[0], block=B, subrate=0.25, method="dd"),
                   dict(d[1], block=B, subrate=0.2, method="zz")]).budget().sense().fetch()
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
        xo, sig = oida.ida(got["y"].astype(np.float64), got["k"], B, img.shape[0], img.shape[1], iters, 2.0)
        di = run.plan.images[i]
        xi = xh[di["out_offset"]:di["out_offset"] + xo.size].reshape(xo.shape)
        assert np.allclose(trh[:, i], sig, rtol=1e-5, atol=0), f"sigma trace, image {i}"
        assert np.max(np.abs(xi - xo)) < 2e-3, f"x error, image {i}"


def test_denoisers_on_block_8_plans():
    """BM3D runs on any image size; the CNN needs W' % 16 == 0 and H' % 8 == 0
    and says so (EUNSUPPORTED) otherwise."""
    import torch
    import paper_2001_09632_amd as g
    from oracle import cnn as ocnn
    dev = device()
    img = synth.synth_image(610, 72, 40)                    # W' = 40: not a multiple of 16
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=8, subrate=0.25, method="dd")]).budget().sense().reconstruct().fetch()
    x = torch.empty(run.plan.pixels, dtype=torch.float32, device=dev)
    ws = torch.empty(g.ida_workspace_bytes(run.plan, "bm3d"), dtype=torch.uint8, device=dev)
    g.ida_refine(run.plan, run.y, run.k, run.off, x, 2, 2.0, "bm3d", workspace=ws)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(x.cpu().numpy()))
    params = torch.from_numpy(g.denoiser_params(ocnn.init_params(1), (0.5, 300.0))).to(dev)
    ws2 = torch.empty(g.ida_workspace_bytes(run.plan, "cnn"), dtype=torch.uint8, device=dev)
    with pytest.raises(g.AbcsError, match="EUNSUPPORTED"):
        g.ida_refine(run.plan, run.y, run.k, run.off, x, 1, 2.0, "cnn", params=params, workspace=ws2)


@pytest.mark.parametrize("B", [8, 32])
def test_short_tiles_every_remainder(B):
    """Block rows of 1 .. 7 blocks and tiles whose block count leaves every
    remainder modulo 4 (the B = 8 kernels transform four blocks at a time),
    both transforms, all three rules, one plan."""
    widths = [B * n for n in (1, 2, 3, 4, 5, 6, 7, 17, 18, 19)]
    imgs = [synth.synth_image(1900 + i, 2 * B + 3, w + (i % 3)) for i, w in enumerate(widths)]
    px, d = pack_images(imgs, pitch_pad=4)
    entries, cases = [], []
    for i, img in enumerate(imgs):
        m = ("zz", "bbv", "dd")[i % 3]
        cr = (0.3, 0.45, 0.2)[i % 3]
        entries.append(dict(d[i], block=B, subrate=cr, method=m, transform="dct"))
        cases.append((i, "dct", m, cr))
        entries.append(dict(d[i], block=B, subrate=cr, method="dd", transform="wht"))
        cases.append((i, "wht", "dd", cr))
    run = Run(px, entries).budget().sense().reconstruct().fetch()
    for j, (i, xf, m, cr) in enumerate(cases):
        img = imgs[i]
        got = run.image(j)
        k, stat = orc.budget(img, B, cr, orc.METHOD_NAMES[m], transform=xf)
        assert np.array_equal(got["k"], k), f"k (entry {j}: {img.shape}, {xf}, {m})"
        assert np.array_equal(got["stat"], stat), f"stat (entry {j})"
        y = orc.sense(img, B, k, transform=xf)
        if y.size:
            assert np.max(np.abs(got["y"] - y)) < Y_TOL[B], f"y (entry {j}: {img.shape}, {xf})"
        rec = orc.reconstruct(got["y"].astype(np.float64), B, k, *img.shape, transform=xf)
        assert np.max(np.abs(got["out"] - rec)) < PX_TOL, f"pixels (entry {j}: {img.shape}, {xf})"
