"""GPU parity of the BBV samples (abcs_bbv_samples) and of IDA with them as
extra difference rows of A (ida_refine_bbv, Section V-A), against the oracle.

Bars: samples bit-exact (integers); IDA with the identity denoiser: x within
2e-3 and sigma within 1e-5 relative of the FP64 oracle, as for plain IDA.
"""
import numpy as np
import pytest

import synth
from oracle import abcs as orc
from oracle import ida as oida

from gpu_util import Run, pack_images, device

pytestmark = pytest.mark.gpu


def _entries():
    sizes = [(64, 80, 16, 0.2), (131, 77, 8, 0.3), (96, 160, 32, 0.15), (256, 256, 16, 0.1), (200, 71, 16, 0.45)]
    imgs = [synth.synth_image(1800 + i, h, w) for i, (h, w, _, _) in enumerate(sizes)]
    px, d = pack_images(imgs, pitch_pad=4)
    entries, cases = [], []
    for i, (h, w, B, cr) in enumerate(sizes):
        for m in ("bbv", "dd"):
            entries.append(dict(d[i], block=B, subrate=cr, method=m))
            cases.append((i, B, cr, m))
    return imgs, px, entries, cases


def test_bbv_samples_match_oracle():
    import torch
    import paper_2001_09632_amd as g
    imgs, px, entries, cases = _entries()
    run = Run(px, entries)
    out = torch.full((max(1, run.plan.bbv_total),), float("nan"), dtype=torch.float32, device=device())
    g.bbv_samples(run.plan, run.px, out)
    torch.cuda.synchronize()
    h = out.cpu().numpy()
    for j, (i, B, cr, m) in enumerate(cases):
        d = run.plan.images[j]
        if m != "bbv":
            assert d["n_bbv"] == 0
            continue
        s = orc.budget_scalars(imgs[i].shape[0], imgs[i].shape[1], B, cr, orc.BBV)
        want = orc.bbv_samples(imgs[i], B, s["L"], s["X0"], s["nS"])
        assert d["n_bbv"] == want.size
        got = h[d["bbv_offset"]:d["bbv_offset"] + d["n_bbv"]]
        assert np.array_equal(got, want.astype(np.float32)), f"samples, entry {j} (B {B}, C_R {cr})"


def test_ida_with_bbv_rows_matches_oracle():
    import torch
    import paper_2001_09632_amd as g
    imgs, px, entries, cases = _entries()
    run = Run(px, entries).budget().sense().fetch()
    dev = device()
    bbv = torch.empty(max(1, run.plan.bbv_total), dtype=torch.float32, device=dev)
    g.bbv_samples(run.plan, run.px, bbv)
    iters = 5
    ws = torch.empty(g.ida_workspace_bytes(run.plan, "identity"), dtype=torch.uint8, device=dev)
    x = torch.full((run.plan.pixels,), float("nan"), dtype=torch.float32, device=dev)
    tr = torch.full((iters * run.plan.n,), float("nan"), dtype=torch.float32, device=dev)
    g.ida_refine_bbv(run.plan, run.y, run.k, run.off, bbv, x, iters, 2.0, "identity", sigma_trace=tr, workspace=ws)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    trh = tr.cpu().numpy().reshape(iters, run.plan.n)
    bh = bbv.cpu().numpy()
    for j, (i, B, cr, m) in enumerate(cases):
        img = imgs[i]
        got = run.image(j)
        d = run.plan.images[j]
        extra = None
        if m == "bbv":
            s = orc.budget_scalars(img.shape[0], img.shape[1], B, cr, orc.BBV)
            samples = bh[d["bbv_offset"]:d["bbv_offset"] + d["n_bbv"]].astype(np.float64)
            extra = (samples, s["L"], s["X0"], s["nS"])
        xo, sig = oida.ida(got["y"].astype(np.float64), got["k"], B, img.shape[0], img.shape[1], iters, 2.0,
                           bbv=extra)
        xi = xh[d["out_offset"]:d["out_offset"] + xo.size].reshape(xo.shape)
        assert np.allclose(trh[:, j], sig, rtol=1e-5, atol=0), f"sigma trace, entry {j} ({m}, B {B})"
        assert np.max(np.abs(xi - xo)) < 2e-3, f"x error {np.max(np.abs(xi - xo))}, entry {j} ({m}, B {B})"


def test_ida_bbv_rows_with_bm3d_runs_and_plain_plan_is_unchanged():
    """A plan without BBV images gives ida_refine's result exactly; with BM3D
    the loop stays finite."""
    import torch
    import paper_2001_09632_amd as g
    img = synth.synth_image(1900, 64, 64)
    px, d = pack_images([img])
    dev = device()
    run = Run(px, [dict(d[0], block=16, subrate=0.25, method="dd")]).budget().sense()
    ws = torch.empty(g.ida_workspace_bytes(run.plan, "identity"), dtype=torch.uint8, device=dev)
    x1 = torch.empty(run.plan.pixels, dtype=torch.float32, device=dev)
    x2 = torch.empty_like(x1)
    g.ida_refine(run.plan, run.y, run.k, run.off, x1, 4, 2.0, "identity", workspace=ws)
    g.ida_refine_bbv(run.plan, run.y, run.k, run.off, None, x2, 4, 2.0, "identity", workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)
    run = Run(px, [dict(d[0], block=16, subrate=0.25, method="bbv")]).budget().sense()
    bbv = torch.empty(run.plan.bbv_total, dtype=torch.float32, device=dev)
    g.bbv_samples(run.plan, run.px, bbv)
    ws = torch.empty(g.ida_workspace_bytes(run.plan, "bm3d"), dtype=torch.uint8, device=dev)
    x = torch.empty(run.plan.pixels, dtype=torch.float32, device=dev)
    g.ida_refine_bbv(run.plan, run.y, run.k, run.off, bbv, x, 3, 2.0, "bm3d", workspace=ws)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(x).all())
