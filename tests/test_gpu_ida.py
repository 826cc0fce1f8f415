"""GPU parity of the IDA transform steps and noise-level estimate
(Section VI; eqs 13, 15, 25, 28) with the identity denoiser, against the FP64
oracle and the closed-form recurrence of a measured coefficient.

Bars: sigma^t within 1e-5 relative; x^T within 2e-3 absolute after up to 8
iterations (each iteration adds one float32 forward and one inverse transform,
each within 1e-3 of exact on [0, 255]-scale data, and with D_F >= 2 the
recurrence damps old errors by sqrt(1/D_F) per step).
"""
import math

import numpy as np
import pytest

import synth
from oracle import abcs as orc
from oracle import ida as oida

from gpu_util import Run, pack_images, device

pytestmark = pytest.mark.gpu

SIG_RTOL = 1e-5
X_TOL = 2e-3


def _run_ida(run, iters, damping, y=None):
    import torch
    import paper_2001_09632_amd as g
    dev = device()
    ws = torch.empty(g.ida_workspace_bytes(run.plan, "identity"), dtype=torch.uint8, device=dev)
    x = torch.full((run.plan.pixels,), float("nan"), dtype=torch.float32, device=dev)
    tr = torch.full((max(1, iters * run.plan.n),), float("nan"), dtype=torch.float32, device=dev)
    g.ida_refine(run.plan, run.y if y is None else y, run.k, run.off, x, iters, damping, "identity",
                 sigma_trace=tr, workspace=ws)
    torch.cuda.synchronize()
    return x.cpu().numpy(), tr.cpu().numpy()[: iters * run.plan.n].reshape(iters, run.plan.n)


def _image_out(run, x, i):
    d = run.plan.images[i]
    hc, wc = d["cropped_height"], d["cropped_width"]
    return x[d["out_offset"]:d["out_offset"] + hc * wc].reshape(hc, wc)


@pytest.mark.parametrize("damping,ratios", [(2.0, [1.0, 1.5, 1.25, 0.875, 0.8125, 0.96875, 1.078125]),
                                            (1.0, [1.0, 2.0, 2.0, 1.0, 0.0, 0.0, 1.0, 2.0]),
                                            (math.inf, [1.0, 1.0, 1.0])])
def test_identity_recurrence_closed_form(damping, ratios):
    img = synth.synth_image(40, 128, 96)
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=16, subrate=0.3, method="dd")]).budget().sense().fetch()
    y = run.image(0)["y"].astype(np.float64)
    k = run.image(0)["k"]
    for t, ratio in enumerate(ratios, start=1):
        x, _ = _run_ida(run, t, damping)
        c = orc.sense_op(_image_out(run, x, 0).astype(np.float64), 16, k)
        assert np.max(np.abs(c - ratio * y)) < 2e-3 * max(1.0, ratio) * 4, f"t={t}"


def test_ida_identity_matches_oracle_mixed_batch():
    sizes = [(128, 128), (96, 160), (64, 64), (200, 136)]
    imgs = [synth.synth_image(50 + i, h, w) for i, (h, w) in enumerate(sizes)]
    crs = [0.1, 0.3, 0.2, 0.25]
    methods = ["bbv", "dd", "zz", "dd"]
    px, d = pack_images(imgs)
    run = Run(px, [dict(d[i], block=16, subrate=crs[i], method=methods[i]) for i in range(4)]).budget().sense() \
        .fetch()
    iters = 8
    x, tr = _run_ida(run, iters, 2.0)
    for i, img in enumerate(imgs):
        got = run.image(i)
        y64 = got["y"].astype(np.float64)
        xo, sig = oida.ida(y64, got["k"], 16, img.shape[0], img.shape[1], iters, 2.0)
        assert np.allclose(tr[:, i], sig, rtol=SIG_RTOL, atol=0), f"sigma trace image {i}"
        err = np.max(np.abs(_image_out(run, x, i) - xo))
        assert err < X_TOL, f"x error {err} image {i}"


def test_ida_first_iterate_is_real_time_decoder():
    img = synth.synth_image(60, 64, 80)
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=16, subrate=0.25, method="bbv")]).budget().sense().reconstruct().fetch()
    x, tr = _run_ida(run, 1, 2.0)
    assert np.max(np.abs(_image_out(run, x, 0) - run.image(0)["out"])) < 1e-3
    y = run.image(0)["y"].astype(np.float64)
    assert abs(tr[0, 0] - math.sqrt(np.sum(y * y) / y.size)) < SIG_RTOL * tr[0, 0]


def test_ida_zero_iterations_and_bad_arguments():
    import torch
    import paper_2001_09632_amd as g
    img = synth.synth_image(61, 32, 32)
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=16, subrate=0.25, method="zz")]).budget().sense().fetch()
    x, _ = _run_ida(run, 0, 2.0)
    assert np.all(np.isnan(x))            # nothing written
    ws = torch.empty(16, dtype=torch.uint8, device=device())
    xx = torch.empty(run.plan.pixels, dtype=torch.float32, device=device())
    with pytest.raises(g.AbcsError):      # workspace too small
        g.ida_refine(run.plan, run.y, run.k, run.off, xx, 3, 2.0, workspace=ws)
    with pytest.raises(g.AbcsError):      # D_F < 1
        g.ida_refine(run.plan, run.y, run.k, run.off, xx, 3, 0.5, workspace=ws)
