"""IDA (Section VI; eqs 13, 15, 25, 28) with real denoisers on the GPU
against the FP64 oracle loop run with the oracle's denoiser, and what the
learned denoiser gains.

Both loops start from the GPU's measurements y (the sensing step has its own
parity tests), so the comparison isolates the loop and its denoiser.

- BM3D (the plain denoiser): a patch distance or hard-threshold decision
  within float32 rounding of its threshold can pick a different (equally
  valid) group, after which the two loops follow slightly different paths.
  Bars after ITERS iterations: sigma^t within SIG_RTOL relative at every
  iteration, |dPSNR| against the clean image within DPSNR_DB, and at least
  PX_FRAC of the pixels within BM3D_PX_TOL (measured: sigma 1e-6, largest
  pixel difference 0.005).
- CNN (shipped weights): the oracle evaluates the network as its
  arithmetic is defined, bfloat16 weights and hidden activations (rounded in
  float64), float64 sums.  The float32 sums move an activation across a
  bfloat16 rounding boundary now and then, and such a flip propagates
  through the remaining layers: the oracle itself, given an input perturbed
  by 1e-7 relative, moves its output by up to 2% of the network's largest
  correction |v - D(v)|.  Bars: sigma^t and dPSNR as for BM3D; per image the
  largest pixel difference within CNN_PX_MAX and the mean within
  CNN_PX_MEAN of the largest correction of the oracle's last iteration.
"""
import os

import numpy as np
import pytest

import synth
from oracle import bm3d as obm3d
from oracle import cnn as ocnn
from oracle import ida as oida
from oracle import metrics

from gpu_util import Run, device, pack_images
from test_gpu_cnn import bf16_round

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2001_09632_amd",
                       "weights", "ida_cnn.npy")
ITERS = 4
SIG_RTOL = 1e-3
DPSNR_DB = 0.05
BM3D_PX_TOL = 1e-2
PX_FRAC = 0.99
CNN_PX_MAX = 0.05
CNN_PX_MEAN = 0.005
GAIN_DB = 0.5


def _encode(images, subrates, methods):
    px, d = pack_images(images)
    ent = [dict(d[i], block=16, subrate=subrates[i], method=methods[i]) for i in range(len(images))]
    return Run(px, ent).budget().sense().reconstruct().fetch()


def _gpu_ida(run, iters, denoiser, params=None):
    import torch
    import paper_2001_09632_amd as g
    dev = device()
    ws = torch.empty(g.ida_workspace_bytes(run.plan, denoiser), dtype=torch.uint8, device=dev)
    x = torch.full((run.plan.pixels,), float("nan"), dtype=torch.float32, device=dev)
    tr = torch.full((iters * run.plan.n,), float("nan"), dtype=torch.float32, device=dev)
    g.ida_refine(run.plan, run.y, run.k, run.off, x, iters, 2.0, denoiser, params=params, sigma_trace=tr,
                 workspace=ws)
    torch.cuda.synchronize()
    x = x.cpu().numpy().astype(np.float64)
    out = []
    for d in run.plan.images:
        hc, wc = d["cropped_height"], d["cropped_width"]
        out.append(x[d["out_offset"]:d["out_offset"] + hc * wc].reshape(hc, wc))
    return out, tr.cpu().numpy().astype(np.float64).reshape(iters, run.plan.n)


def cnn_bf16_denoiser(params):
    """The learned denoiser as its arithmetic is defined: weights and hidden
    activations rounded to bfloat16, sums in float64; an image whose sigma
    lies outside the accepted range (the last two parameters) goes to BM3D."""
    blob, (lo, hi) = params[:-2], params[-2:]
    layers = [(bf16_round(w), b) for w, b in ocnn.unpack(blob)]

    def denoise(v, sigma):
        if not (lo <= sigma <= hi):
            return obm3d.bm3d(v, sigma)
        a = ocnn.network_input(np.asarray(v)[None], [sigma])
        for i, (w, b) in enumerate(layers):
            a = ocnn.conv3x3(a, w, b)
            if i < len(layers) - 1:
                a = bf16_round(np.maximum(a, 0.0))
        return np.asarray(v, dtype=np.float64) - 255.0 * a[0, ..., 0]

    return denoise


def _compare(run, images, x_gpu, tr_gpu, denoiser, learned):
    for i, img in enumerate(images):
        got = run.image(i)
        h, w = img.shape
        trace = []
        xo, sig = oida.ida(got["y"].astype(np.float64), got["k"], 16, h, w, ITERS, 2.0, denoiser=denoiser,
                           trace=trace)
        rel = np.abs(tr_gpu[:, i] - np.asarray(sig)) / np.asarray(sig)
        diff = np.abs(x_gpu[i] - xo)
        clean = img.astype(np.float64)[: xo.shape[0], : xo.shape[1]]
        dpsnr = metrics.psnr(x_gpu[i], clean) - metrics.psnr(xo, clean)
        corr = float(np.max(np.abs(trace[-1][1] - xo)))
        print(f"image {i}: sigma rel {rel.max():.2e}, max |dx| {diff.max():.4f}, mean {diff.mean():.4f}, "
              f"largest correction {corr:.2f}, dPSNR {dpsnr:+.4f} dB")
        assert rel.max() < SIG_RTOL, (i, rel)
        assert abs(dpsnr) < DPSNR_DB, (i, dpsnr)
        if learned:
            assert diff.max() <= CNN_PX_MAX * corr and diff.mean() <= CNN_PX_MEAN * corr, (i, diff.max(), corr)
        else:
            assert np.mean(diff <= BM3D_PX_TOL) >= PX_FRAC, (i, np.mean(diff <= BM3D_PX_TOL))


def test_ida_bm3d_matches_oracle():
    images = [synth.synth_image(2200, 64, 64), synth.synth_image(2201, 48, 80)]
    run = _encode(images, [0.15, 0.25], ["dd", "bbv"])
    x, tr = _gpu_ida(run, ITERS, "bm3d")
    _compare(run, images, x, tr, obm3d.bm3d, False)


def test_ida_cnn_matches_oracle():
    import torch
    params = np.load(WEIGHTS)
    images = [synth.synth_image(2202, 64, 64), synth.synth_image(2203, 48, 80)]
    run = _encode(images, [0.2, 0.3], ["bbv", "dd"])
    x, tr = _gpu_ida(run, ITERS, "cnn", torch.from_numpy(params).to(device()))
    _compare(run, images, x, tr, cnn_bf16_denoiser(params.astype(np.float64)), True)


def test_learned_ida_gain_on_held_out_images():
    """The shipped network (trained on crops of images with seeds 10000 and
    up) on the 16 256 x 256 images of the IDA evaluation batch (seeds
    2000-2015, C_R ~ U(0.1, 0.3) from stream seed 3, DD on even and BBV on
    odd images): learned IDA at 15 iterations must beat the real-time decoder
    I_o by GAIN_DB and come within 0.1 dB of plain BM3D IDA at 30 iterations,
    the gain the learned denoiser exists for."""
    import torch
    seeds = list(range(2000, 2016))
    crs = np.random.default_rng(3).uniform(0.1, 0.3, size=32)[:16]
    images = [synth.synth_image(s, 256, 256) for s in seeds]
    run = _encode(images, list(crs), ["dd" if i % 2 == 0 else "bbv" for i in range(16)])
    prm = torch.from_numpy(np.load(WEIGHTS).astype(np.float32)).to(device())
    x_cnn, _ = _gpu_ida(run, 15, "cnn", prm)
    x_bm3d, _ = _gpu_ida(run, 30, "bm3d")
    p_io = np.array([metrics.psnr(run.image(i)["out"], im) for i, im in enumerate(images)])
    p_cnn = np.array([metrics.psnr(x, im) for x, im in zip(x_cnn, images)])
    p_bm3d = np.array([metrics.psnr(x, im) for x, im in zip(x_bm3d, images)])
    for i in range(16):
        print(f"image {i} (C_R {crs[i]:.3f}): I_o {p_io[i]:.2f}, learned {p_cnn[i]:.2f}, plain {p_bm3d[i]:.2f} dB")
    print(f"mean PSNR: I_o {p_io.mean():.3f}, learned IDA {p_cnn.mean():.3f}, plain IDA {p_bm3d.mean():.3f} dB")
    assert p_cnn.mean() > p_io.mean() + GAIN_DB
    assert p_cnn.mean() >= p_bm3d.mean() - 0.1
