"""GPU parity of DnCNN-17 with batch normalisation (Section VI-4) against the
FP64 oracle: inference (normalisation folded into the convolutions) and one
training step (batch statistics, gradients of every parameter, running
statistics, Adam).

The oracle runs with the weights rounded to bfloat16 and, where the kernels
store them in bfloat16, with the activations and pre-normalisation values
rounded too; the remaining difference is rounding order (float32 sums) and
the bfloat16 rounding of the folded weights and of the gradients between
layers.  Bars: network output within 5% of the largest |f| (1% on average);
loss within 1%; per-layer gradients within twice the oracle's own rounding
noise floor plus 0.05 (relative); running statistics within 1e-3 relative.
"""
import numpy as np
import pytest

import synth
from oracle import cnn as ocnn
from oracle import dncnn

from gpu_util import device
from test_gpu_cnn import bf16_round

pytestmark = pytest.mark.gpu


def _blob(seed):
    blob = dncnn.init_params(seed)
    w1, b1, mids, w17, b17 = dncnn.unpack(blob)
    rng = np.random.default_rng(seed)
    w17 *= 10.0
    b1[:] = rng.normal(0, 0.05, size=b1.shape)
    for _, g, b in mids:
        g[:] = rng.uniform(0.6, 1.4, size=g.shape)
        b[:] = rng.normal(0, 0.1, size=b.shape)
    return blob


def _rounded(blob):
    w1, b1, mids, w17, b17 = dncnn.unpack(blob)
    return dncnn.pack(bf16_round(w1), b1, [(bf16_round(w), g, b) for w, g, b in mids], bf16_round(w17), b17)


def _plan(n, h, w):
    import paper_2001_09632_amd as g
    return g.Plan([dict(height=h, width=w, block=16, subrate=0.25, method="zz", pixel_offset=0) for _ in range(n)])


def _put(plan, arrs):
    import torch
    t = torch.zeros(plan.pixels, dtype=torch.float32, device=device())
    for i, a in enumerate(arrs):
        o = plan.images[i]["out_offset"]
        t[o:o + a.size] = torch.from_numpy(a.astype(np.float32).reshape(-1)).to(device())
    return t


def _folded_forward_bf16(blob, running, v, sigma):
    """The inference network as the kernels evaluate it: folded weights and
    the first / last layers rounded to bfloat16, activations rounded."""
    w1, b1, mids, w17, b17 = dncnn.fold(blob, running)
    a = bf16_round(np.maximum(ocnn.conv3x3(ocnn.network_input(v, sigma), bf16_round(w1), b1), 0.0))
    for w, b in mids:
        a = bf16_round(np.maximum(ocnn.conv3x3(a, bf16_round(w), b), 0.0))
    return np.asarray(v, dtype=np.float64) - 255.0 * ocnn.conv3x3(a, bf16_round(w17), b17)[..., 0]


def test_dncnn_inference_matches_oracle():
    import torch
    import paper_2001_09632_amd as g
    assert g.dncnn_param_count() == dncnn.param_count() and g.dncnn_running_count() == dncnn.running_count()
    blob = _blob(21)
    rng = np.random.default_rng(22)
    run = np.concatenate([np.concatenate([rng.normal(0, 0.2, 64), rng.uniform(0.3, 2.0, 64)]) for _ in range(15)])
    imgs = [synth.synth_image(200 + i, 32, 48).astype(np.float64) for i in range(2)]
    sig = [25.0, 300.0]
    plan = _plan(2, 32, 48)
    xin = _put(plan, imgs)
    out = torch.full_like(xin, float("nan"))
    prm = torch.from_numpy(np.concatenate([blob, run]).astype(np.float32)).to(device())
    ws = torch.empty(g.denoise_workspace_bytes(plan, "dncnn"), dtype=torch.uint8, device=device())
    g.denoise(plan, xin, torch.tensor(sig, dtype=torch.float32, device=device()), out, "dncnn", params=prm,
              workspace=ws)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for i, im in enumerate(imgs):
        got = o[plan.images[i]["out_offset"]:plan.images[i]["out_offset"] + im.size].reshape(im.shape)
        ref = _folded_forward_bf16(blob, run, im[None], [sig[i]])[0]
        exact = dncnn.forward(blob, im[None], [sig[i]], running=run, train=False)[0]
        f = np.abs(im - exact) / 255.0
        err = np.abs(got - ref) / 255.0
        assert err.max() < 0.05 * f.max() and err.mean() < 0.01 * f.max(), (i, err.max(), err.mean(), f.max())


def _train(blob, imgs, tgts, sig, lr=0.0, step=1):
    import torch
    import paper_2001_09632_amd as g
    plan = _plan(len(imgs), *imgs[0].shape)
    dev = device()
    n = len(blob)
    st = dict(prm=torch.from_numpy(blob.astype(np.float32)).to(dev), m=torch.zeros(n, device=dev),
              v=torch.zeros(n, device=dev), loss=torch.zeros(1, device=dev), grad=torch.zeros(n, device=dev),
              run=torch.from_numpy(dncnn.init_running().astype(np.float32)).to(dev))
    ws = torch.empty(g.dncnn_train_workspace_bytes(plan), dtype=torch.uint8, device=dev)
    g.dncnn_train_step(plan, st["prm"], st["m"], st["v"], st["run"], step, lr, _put(plan, imgs),
                       torch.tensor(sig, dtype=torch.float32, device=dev), _put(plan, tgts), st["loss"], st["grad"],
                       workspace=ws)
    torch.cuda.synchronize()
    return {k: t.cpu().numpy().astype(np.float64) for k, t in st.items()}


def test_dncnn_training_step_matches_oracle():
    """Gradients through 15 normalisations amplify rounding: the oracle itself,
    with the inputs of its bfloat16 roundings perturbed by 1e-6 relative (a
    few roundings in 10^4 flip), moves the first layer's gradient by ~0.4
    relative.  The bar per parameter group is twice that noise floor plus
    0.05, which at the last layers (floor ~0) means 5%."""
    blob = _blob(23)
    rng = np.random.default_rng(24)
    imgs = [synth.synth_image(210 + i, 32, 32).astype(np.float64) for i in range(3)]
    tgts = [np.clip(im + rng.normal(0, 15, im.shape), 0, 255) for im in imgs]
    sig = [20.0, 60.0, 35.0]
    got = _train(blob, imgs, tgts, sig)
    rb = _rounded(blob)
    l_ref, g_ref, stats = dncnn.loss_and_grad(rb, np.stack(imgs), sig, np.stack(tgts), round_act=bf16_round,
                                              round_grad=bf16_round)
    pr = np.random.default_rng(5)

    def perturbed(x):
        return bf16_round(x * (1 + 1e-6 * pr.standard_normal(np.shape(x))))

    _, g_floor, _ = dncnn.loss_and_grad(rb, np.stack(imgs), sig, np.stack(tgts), round_act=perturbed,
                                        round_grad=perturbed)
    assert abs(got["loss"][0] - l_ref) < 1e-2 * l_ref, (got["loss"][0], l_ref)
    w1o, b1o, mid0, w17o, b17o, total = dncnn.offsets()
    pieces = [("W1", 0, b1o), ("b1", b1o, mid0)]
    for m in range(15):
        o = mid0 + m * dncnn.MID_STRIDE
        pieces += [(f"W{m + 2}", o, o + 36864), (f"gamma{m + 2}", o + 36864, o + 36928),
                   (f"beta{m + 2}", o + 36928, o + dncnn.MID_STRIDE)]
    pieces += [("W17", w17o, b17o), ("b17", b17o, total)]
    for name, a0, a1 in pieces:
        b = g_ref[a0:a1]
        rel = float(np.linalg.norm(got["grad"][a0:a1] - b) / (np.linalg.norm(b) + 1e-30))
        floor = float(np.linalg.norm(g_floor[a0:a1] - b) / (np.linalg.norm(b) + 1e-30))
        assert rel < 2.0 * floor + 0.05, (name, rel, floor)
    run_ref = dncnn.update_running(dncnn.init_running(), stats)
    assert np.allclose(got["run"], run_ref, rtol=1e-3, atol=1e-4)


def test_dncnn_adam_and_loss_decrease():
    import torch
    import paper_2001_09632_amd as g
    blob = _blob(25)
    rng = np.random.default_rng(26)
    clean = [synth.synth_image(220 + i, 32, 32).astype(np.float64) for i in range(4)]
    noisy = [c + rng.normal(0, 20, c.shape) for c in clean]
    plan = _plan(4, 32, 32)
    dev = device()
    n = len(blob)
    prm = torch.from_numpy(blob.astype(np.float32)).to(dev)
    m, v = torch.zeros(n, device=dev), torch.zeros(n, device=dev)
    run = torch.from_numpy(dncnn.init_running().astype(np.float32)).to(dev)
    loss, grad = torch.zeros(1, device=dev), torch.zeros(n, device=dev)
    ws = torch.empty(g.dncnn_train_workspace_bytes(plan), dtype=torch.uint8, device=dev)
    x, t = _put(plan, noisy), _put(plan, clean)
    sig = torch.full((4,), 20.0, device=dev)
    p0 = prm.cpu().numpy().astype(np.float64)
    g.dncnn_train_step(plan, prm, m, v, run, 1, 1e-3, x, sig, t, loss, grad, workspace=ws)
    torch.cuda.synchronize()
    l0 = float(loss.cpu()[0])
    exp, _, _ = dncnn.adam_step(p0, np.zeros(n), np.zeros(n), grad.cpu().numpy().astype(np.float64), 1, 1e-3)
    assert np.max(np.abs(prm.cpu().numpy() - exp)) < 1e-6
    for step in range(2, 61):
        g.dncnn_train_step(plan, prm, m, v, run, step, 1e-3, x, sig, t, loss, None, workspace=ws)
    torch.cuda.synchronize()
    assert float(loss.cpu()[0]) < 0.7 * l0


def test_ida_with_dncnn_denoiser_runs():
    import torch
    import paper_2001_09632_amd as g
    from gpu_util import Run, pack_images
    img = synth.synth_image(230, 64, 64)
    px, d = pack_images([img])
    run = Run(px, [dict(d[0], block=16, subrate=0.25, method="dd")]).budget().sense()
    prm = torch.from_numpy(np.concatenate([_blob(27), dncnn.init_running()]).astype(np.float32)).to(device())
    ws = torch.empty(g.ida_workspace_bytes(run.plan, "dncnn"), dtype=torch.uint8, device=device())
    x = torch.empty(run.plan.pixels, dtype=torch.float32, device=device())
    g.ida_refine(run.plan, run.y, run.k, run.off, x, 3, 2.0, "dncnn", params=prm, workspace=ws)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(x).all())
