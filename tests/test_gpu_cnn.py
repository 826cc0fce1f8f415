"""GPU parity of the learned denoiser (8-layer CNN, bfloat16 weights and
activations, float32 sums) against the FP64 oracle.

The oracle runs with the same weights rounded to bfloat16, so the remaining
difference is the bfloat16 rounding of the seven stored activations (relative
2^-9 each, accumulating over depth): the bar is 3% of the largest |f| for the
network output f and 0.5% on average.
"""
import numpy as np
import pytest

import synth
from oracle import cnn as ocnn

from gpu_util import device

pytestmark = pytest.mark.gpu


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _gpu_forward(images, sigmas, blob):
    import torch
    import paper_2001_09632_amd as g
    dev = device()
    plan = g.Plan([dict(height=im.shape[0], width=im.shape[1], block=16, subrate=0.25, method="zz",
                        pixel_offset=0) for im in images])
    xin = torch.zeros(plan.pixels, dtype=torch.float32, device=dev)
    for i, im in enumerate(images):
        d = plan.images[i]
        xin[d["out_offset"]:d["out_offset"] + im.size] = torch.from_numpy(im.astype(np.float32).reshape(-1)).to(dev)
    sig = torch.tensor(sigmas, dtype=torch.float32, device=dev)
    prm = torch.from_numpy(blob.astype(np.float32)).to(dev)
    out = torch.full_like(xin, float("nan"))
    ws = torch.empty(g.denoise_workspace_bytes(plan, "cnn"), dtype=torch.uint8, device=dev)
    g.denoise(plan, xin, sig, out, "cnn", params=prm, workspace=ws)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return [o[plan.images[i]["out_offset"]:plan.images[i]["out_offset"] + im.size].reshape(im.shape)
            for i, im in enumerate(images)]


def _blob(seed):
    blob = ocnn.init_params(seed)
    layers = ocnn.unpack(blob)
    layers[-1][0][:] *= 10.0   # make f matter
    rng = np.random.default_rng(seed)
    for w, b in layers:
        b[:] = rng.normal(0, 0.05, size=b.shape)
    return ocnn.pack(layers)


def test_cnn_forward_matches_oracle():
    assert __import__("paper_2001_09632_amd").cnn_param_count() == ocnn.param_count()
    blob = _blob(11)
    imgs = [synth.synth_image(100, 32, 48).astype(np.float64), synth.synth_image(101, 16, 16).astype(np.float64)]
    sig = [25.0, 400.0]
    got = _gpu_forward(imgs, sig, blob)
    rb = ocnn.pack([(bf16_round(w), b) for w, b in ocnn.unpack(blob)])
    for i, im in enumerate(imgs):
        ref = ocnn.forward(rb, im[None], [sig[i]])[0]
        f = (im - ref) / 255.0
        err = np.abs(got[i] - ref) / 255.0
        assert err.max() < 0.03 * np.abs(f).max() and err.mean() < 0.005 * np.abs(f).max(), \
            (i, err.max(), err.mean(), np.abs(f).max())


def test_cnn_zero_last_layer_is_identity():
    blob = _blob(12)
    layers = ocnn.unpack(blob)
    layers[-1][0][:] = 0.0
    layers[-1][1][:] = 0.0
    im = synth.synth_image(102, 32, 32).astype(np.float64)
    got = _gpu_forward([im], [30.0], ocnn.pack(layers))[0]
    assert np.array_equal(got, im.astype(np.float32))
