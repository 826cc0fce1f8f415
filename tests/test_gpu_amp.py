"""D-AMP and DAMP-D (eqs 14, 24, 27) on the GPU against the FP64 oracle.

Identity denoiser: sigma and alpha traces within 1e-4 relative and iterates
within 1e-3 of their own magnitude (with D-AMP's alpha ~ n / m > 1 the
coefficients grow geometrically, as the paper reports for D-AMP on this
deterministic sensing operator).  BM3D: the loop runs, the Monte-Carlo
alpha lies in [0, 1.5 n / m] and repeated runs are bit-identical."""
import numpy as np
import pytest

import synth
from oracle import ida as oida

from gpu_util import Run, pack_images, device

pytestmark = pytest.mark.gpu


def _setup():
    imgs = [synth.synth_image(800, 64, 64), synth.synth_image(801, 48, 80)]
    px, d = pack_images(imgs)
    run = Run(px, [dict(d[0], block=16, subrate=0.25, method="dd"),
                   dict(d[1], block=16, subrate=0.3, method="bbv")]).budget().sense().fetch()
    probe = np.random.default_rng(9).standard_normal(run.plan.pixels).astype(np.float32)
    return imgs, run, probe


def _amp_gpu(run, probe, iters, algorithm, damping, denoiser):
    import torch
    import paper_2001_09632_amd as g
    dev = device()
    x = torch.full((run.plan.pixels,), float("nan"), dtype=torch.float32, device=dev)
    st = torch.full((iters * run.plan.n,), float("nan"), dtype=torch.float32, device=dev)
    at = torch.full((iters * run.plan.n,), float("nan"), dtype=torch.float32, device=dev)
    ws = torch.empty(g.amp_workspace_bytes(run.plan, denoiser), dtype=torch.uint8, device=dev)
    b = torch.from_numpy(probe).to(dev)
    g.amp_refine(run.plan, run.y, run.k, run.off, x, iters, b, damping=damping, algorithm=algorithm,
                 denoiser=denoiser, sigma_trace=st, alpha_trace=at, workspace=ws)
    torch.cuda.synchronize()
    n = run.plan.n
    return x.cpu().numpy(), st.cpu().numpy().reshape(iters, n), at.cpu().numpy().reshape(iters, n)


@pytest.mark.parametrize("algorithm,damping,iters", [("damp", 2.0, 4), ("damp-d", 8.0, 6)])
def test_amp_identity_matches_oracle(algorithm, damping, iters):
    imgs, run, probe = _setup()
    x, st, at = _amp_gpu(run, probe, iters, algorithm, damping, "identity")
    for i, img in enumerate(imgs):
        d = run.plan.images[i]
        got = run.image(i)
        hw = d["cropped_height"] * d["cropped_width"]
        b = probe[d["out_offset"]:d["out_offset"] + hw].astype(np.float64).reshape(img.shape)
        xo, so, ao = oida.amp(got["y"].astype(np.float64), got["k"], 16, img.shape[0], img.shape[1], iters,
                              damping, b, algorithm=algorithm)
        assert np.allclose(st[:, i], so, rtol=1e-4, atol=0), f"sigma trace, image {i}"
        assert at[0, i] == 0.0 and np.allclose(at[1:, i], ao[1:], rtol=1e-4, atol=0), f"alpha trace, image {i}"
        xi = x[d["out_offset"]:d["out_offset"] + hw].reshape(img.shape)
        assert np.max(np.abs(xi - xo)) <= 1e-3 * max(1.0, float(np.max(np.abs(xo)))), f"x, image {i}"


def test_amp_bm3d_runs_and_repeats():
    imgs, run, probe = _setup()
    x1, s1, a1 = _amp_gpu(run, probe, 3, "damp-d", 2.0, "bm3d")
    x2, s2, a2 = _amp_gpu(run, probe, 3, "damp-d", 2.0, "bm3d")
    assert np.all(np.isfinite(x1)) and np.array_equal(x1, x2) and np.array_equal(a1, a2)
    for i in range(run.plan.n):
        d = run.plan.images[i]
        ratio = d["cropped_height"] * d["cropped_width"] / d["n_meas"]
        assert np.all(a1[1:, i] >= 0.0) and np.all(a1[1:, i] <= 1.5 * ratio / 2.0), f"alpha {a1[:, i]}"


def test_amp_arguments():
    import torch
    import paper_2001_09632_amd as g
    imgs, run, probe = _setup()
    dev = device()
    x = torch.empty(run.plan.pixels, dtype=torch.float32, device=dev)
    ws = torch.empty(g.amp_workspace_bytes(run.plan, "identity"), dtype=torch.uint8, device=dev)
    with pytest.raises(g.AbcsError, match="EINVAL"):
        g.amp_refine(run.plan, run.y, run.k, run.off, x, 2, None, workspace=ws)          # no probe
    b = torch.from_numpy(probe).to(dev)
    with pytest.raises(g.AbcsError, match="EINVAL"):
        g.amp_refine(run.plan, run.y, run.k, run.off, x, 2, b, algorithm=0, workspace=ws)
    with pytest.raises(g.AbcsError, match="ENOSPACE"):
        g.amp_refine(run.plan, run.y, run.k, run.off, x, 2, b, workspace=ws[:16])
