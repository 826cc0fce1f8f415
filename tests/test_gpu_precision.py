"""The 16-bit operand modes of the DCT transforms (B = 8, 16, 32) against the
FP64 oracle.

Budgets never depend on the mode.  Bars, for B = 16 and scaled by B / 16 for
the other block sizes (the largest coefficient, the DC of a white block, is
255 B): the compensated modes (BF16x3, FP16x3) keep decoded pixels within
2e-2 of the oracle's decoding of the same measurements and y within 5e-2
(bf16: 16 significant bits per split operand, coefficients up to 4080 at
B = 16); the single-pass modes are data points, checked for bounded error (y
within 1 % of the coefficient range, PSNR of the decoded image within 1 dB of
the float32 path, or above 60 - 20 log10(scale) dB where the float32 path is
near lossless: a single rounding of the coefficients costs about that)."""
import numpy as np
import pytest

import synth
from oracle import abcs as orc

from gpu_util import pack_images, device

pytestmark = pytest.mark.gpu

MODES = ["fp32", "bf16x3", "fp16x3", "bf16", "fp16"]
Y_TOL = {"fp32": 1e-2, "bf16x3": 5e-2, "fp16x3": 1e-2}
PX_TOL = {"fp32": 1e-3, "bf16x3": 2e-2, "fp16x3": 2e-2}


def _run(mode, imgs, entries):
    import torch
    import paper_2001_09632_amd as g
    dev = device()
    px, _ = pack_images(imgs)
    plan = g.Plan(entries)
    pxd = torch.from_numpy(px).to(dev)
    k = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    off = torch.empty(plan.blocks, dtype=torch.int64, device=dev)
    st = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    y = torch.empty(max(1, plan.meas), dtype=torch.float32, device=dev)
    out = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    g.budget(plan, pxd, k, off, st)
    g.sense(plan, pxd, k, off, y, precision=mode)
    g.reconstruct(plan, y, k, off, out, precision=mode)
    torch.cuda.synchronize()
    return plan, k.cpu().numpy(), y.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("B", [8, 16, 32])
@pytest.mark.parametrize("mode", MODES)
def test_precision_modes(mode, B):
    imgs = [synth.synth_image(700 + i, h, w) for i, (h, w) in enumerate([(256, 256), (128, 208)])]
    _, d = pack_images(imgs)
    cases = [(0, 0.25, "dd"), (0, 0.1, "bbv"), (1, 0.5, "zz"), (1, 1.0, "dd")]
    entries = [dict(d[i], block=B, subrate=cr, method=m) for i, cr, m in cases]
    scale = max(1.0, B / 16)
    plan, k, y, out = _run(mode, imgs, entries)
    _, k32, y32, out32 = _run("fp32", imgs, entries) if mode != "fp32" else (plan, k, y, out)
    assert np.array_equal(k, k32)
    for j, (i, cr, m) in enumerate(cases):
        im = plan.images[j]
        img = imgs[i]
        nb = (im["cropped_height"] // B) * (im["cropped_width"] // B)
        kk = k[im["block_offset"]:im["block_offset"] + nb]
        kref, _ = orc.budget(img, B, cr, orc.METHOD_NAMES[m])
        assert np.array_equal(kk, kref)
        yy = y[im["meas_offset"]:im["meas_offset"] + im["n_meas"]]
        yref = orc.sense(img, B, kref)
        hc, wc = im["cropped_height"], im["cropped_width"]
        xo = out[im["out_offset"]:im["out_offset"] + hc * wc].reshape(hc, wc)
        rec = orc.reconstruct(yy.astype(np.float64), B, kref, *img.shape)
        img = img[:hc, :wc]
        yerr = float(np.max(np.abs(yy - yref)))
        perr = float(np.max(np.abs(xo - rec)))
        if mode in Y_TOL:
            assert yerr < Y_TOL[mode] * scale, f"{mode}, B {B}: y error {yerr} (case {j})"
            assert perr < PX_TOL[mode] * scale, f"{mode}, B {B}: pixel error {perr} (case {j})"
        else:
            assert yerr < 0.01 * 255 * B, f"{mode}, B {B}: y error {yerr} (case {j})"
            x32 = out32[im["out_offset"]:im["out_offset"] + hc * wc].reshape(hc, wc)
            p32 = 10 * np.log10(255.0 ** 2 / np.mean((np.clip(x32, 0, 255) - img) ** 2))
            pm = 10 * np.log10(255.0 ** 2 / max(np.mean((np.clip(xo, 0, 255) - img) ** 2), 1e-12))
            assert pm > min(p32, 60.0 - 20 * np.log10(scale)) - 1.0, f"{mode}, B {B}: PSNR {pm:.2f} vs float32 {p32:.2f} (case {j})"
        print(f"B {B} {mode} case {j}: max |dy| {yerr:.2e}, max |dpx| {perr:.2e}")


def test_bad_precision():
    import torch
    import paper_2001_09632_amd as g
    dev = device()
    img = synth.synth_image(710, 64, 64)
    px, d = pack_images([img])
    plan = g.Plan([dict(d[0], block=16, subrate=0.25, method="zz")])
    pxd = torch.from_numpy(px).to(dev)
    k = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    off = torch.empty(plan.blocks, dtype=torch.int64, device=dev)
    st = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    y = torch.empty(plan.meas, dtype=torch.float32, device=dev)
    g.budget(plan, pxd, k, off, st)
    with pytest.raises(g.AbcsError, match="EINVAL"):
        g.sense(plan, pxd, k, off, y, precision=9)
