"""GPU parity of the BM3D denoiser against the FP64 oracle.

On integer-valued inputs the stage-1 patch distances are exact in float32 and
groups match the oracle's; a hard-threshold decision or a stage-2 grouping can
still flip where a value sits within float32 rounding of its threshold, so
parity is stated as: >= 99.5% of pixels within 1e-3 of the oracle, and image
PSNR against the clean image within 0.05 dB.  sigma = 0 and constant images
are exact; runs are bit-identical.
"""
import numpy as np
import pytest

import synth
from oracle import bm3d as obm3d
from oracle import metrics

from gpu_util import device

pytestmark = pytest.mark.gpu


def _denoise(images, sigmas):
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
    out = torch.full_like(xin, float("nan"))
    ws = torch.empty(max(1, g.denoise_workspace_bytes(plan, "bm3d")), dtype=torch.uint8, device=dev)
    g.denoise(plan, xin, sig, out, "bm3d", workspace=ws)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    res = []
    for i, im in enumerate(images):
        d = plan.images[i]
        res.append(o[d["out_offset"]:d["out_offset"] + im.size].reshape(im.shape))
    return res


def _compare(got, ref, clean):
    diff = np.abs(got - ref)
    frac = np.mean(diff > 1e-3)
    dpsnr = abs(metrics.psnr(got, clean) - metrics.psnr(ref, clean))
    return frac, dpsnr, diff.max()


def test_bm3d_integer_input_matches_oracle():
    clean = synth.synth_image(70, 64, 64).astype(np.float64)
    rng = np.random.default_rng(5)
    noisy = np.clip(np.rint(clean + rng.normal(0, 20, clean.shape)), 0, 255)
    got = _denoise([noisy], [20.0])[0]
    ref = obm3d.bm3d(noisy, 20.0)
    frac, dpsnr, mx = _compare(got, ref, clean)
    assert frac <= 0.005 and dpsnr < 0.05, (frac, dpsnr, mx)


def test_bm3d_batch_of_sizes_and_sigmas():
    shapes = [(48, 64), (64, 48), (32, 32)]
    sigmas = [10.0, 35.0, 300.0]
    rng = np.random.default_rng(6)
    cleans = [synth.synth_image(80 + i, h, w).astype(np.float64) for i, (h, w) in enumerate(shapes)]
    noisy = [c + rng.normal(0, min(s, 40.0), c.shape) for c, s in zip(cleans, sigmas)]
    got = _denoise(noisy, sigmas)
    for i in range(3):
        ref = obm3d.bm3d(noisy[i], sigmas[i])
        frac, dpsnr, mx = _compare(got[i], ref, cleans[i])
        assert frac <= 0.005 and dpsnr < 0.05, (i, frac, dpsnr, mx)


def test_bm3d_sigma_zero_constant_and_repeatable():
    rng = np.random.default_rng(7)
    a = rng.uniform(0, 255, (32, 48))
    c = np.full((32, 32), 100.0)
    out = _denoise([a, c], [0.0, 20.0])
    assert np.array_equal(out[0], a.astype(np.float32))
    assert np.ptp(out[1]) < 1e-4 and abs(out[1][0, 0] - obm3d.bm3d(c, 20.0)[0, 0]) < 1e-3
    x = synth.synth_image(90, 48, 48).astype(np.float64) + rng.normal(0, 15, (48, 48))
    o1 = _denoise([x], [15.0])[0]
    o2 = _denoise([x], [15.0])[0]
    assert np.array_equal(o1, o2)


# Validity of the pixels where the GPU and the oracle differ (several results
# are correct where a decision sits within float32 rounding of its
# threshold).  A float32 3-D spectrum value of a group of 8 x 8 patches of
# values in [0, 255] is within EPS_C of the float64 one, and a float32 patch
# distance (mean of 64 squared differences of float32 values, at most a few
# hundred near the stage-2 threshold) within EPS_D.
EPS_C = 0.02
EPS_D = 5e-3


def _denoise_keep(image, sigma):
    """GPU BM3D of one image; returns (output, stage-1 estimate, stage-2
    groups as lists of (y, x) per reference in raster order)."""
    import torch
    import paper_2001_09632_amd as g
    dev = device()
    h, w = image.shape
    plan = g.Plan([dict(height=h, width=w, block=16, subrate=0.25, method="zz", pixel_offset=0)])
    xin = torch.from_numpy(image.astype(np.float32).reshape(-1)).to(dev)
    out = torch.full_like(xin, float("nan"))
    ws = torch.empty(g.denoise_workspace_bytes(plan, "bm3d"), dtype=torch.uint8, device=dev)
    g.denoise(plan, xin, torch.tensor([sigma], dtype=torch.float32, device=dev), out, "bm3d", workspace=ws)
    torch.cuda.synchronize()
    wsh = ws.cpu().numpy()
    go, gb = g.workspace_part(plan, "bm3d", "groups")
    bo, bb = g.workspace_part(plan, "bm3d", "basic")
    basic = wsh[bo:bo + bb].view(np.float32).astype(np.float64).reshape(h, w)
    groups = wsh[go:go + gb].view(np.int32).reshape(-1, obm3d.N2_WIE + 1)
    ry, rx = obm3d.ref_positions(h), obm3d.ref_positions(w)
    gl = []
    for i in range(len(ry)):
        for j in range(len(rx)):
            row = groups[i * len(rx) + j]
            gl.append([(int(q) // w, int(q) % w) for q in row[1:1 + row[0]]])
    return out.cpu().numpy().astype(np.float64).reshape(h, w), basic, gl


def _cover(mask, positions):
    for (py, px) in positions:
        mask[py:py + obm3d.N1, px:px + obm3d.N1] = True


def _sorted_candidates(img, ry, rx):
    """(distance, raster index, (y, x)) of every candidate patch in the
    reference's search window but the reference, by the oracle's order."""
    H, W = img.shape
    N1, hw = obm3d.N1, obm3d.HALF_WIN
    ref = img[ry:ry + N1, rx:rx + N1]
    c = []
    for qy in range(max(0, ry - hw), min(H - N1, ry + hw) + 1):
        for qx in range(max(0, rx - hw), min(W - N1, rx + hw) + 1):
            if (qy, qx) != (ry, rx):
                c.append((float(np.sum((img[qy:qy + N1, qx:qx + N1] - ref) ** 2)) / 64.0, qy * W + qx, (qy, qx)))
    c.sort()
    return c


def _ambiguous_match(img, ry, rx, tau, n2):
    """True when the oracle's group could change under float32 distances:
    a candidate within EPS_D of tau, or two candidates among the first n2
    (plus the next one) whose distances lie within EPS_D of each other."""
    c = _sorted_candidates(img, ry, rx)
    if any(abs(d - tau) <= EPS_D for d, _, _ in c):
        return True
    head = [d for d, _, _ in c if d <= tau + EPS_D][: n2]
    return any(b - a <= EPS_D for a, b in zip(head, head[1:]))


def test_bm3d_differences_come_from_float32_near_ties():
    """Stage 1 on integer input: the matching is exact in float32, so the
    groups are the oracle's and a stage-1 pixel may differ by more than 1e-3
    only inside a group holding a 3-D coefficient within EPS_C of the hard
    threshold.  Stage 2 is compared on the GPU's own stage-1 estimate: each
    reference's group must equal the oracle's member for member unless the
    match is ambiguous in float32, and an output pixel may differ by more
    than 1e-3 only inside such a group."""
    clean = synth.synth_image(71, 64, 64).astype(np.float64)
    rng = np.random.default_rng(8)
    sigma = 25.0
    noisy = np.clip(np.rint(clean + rng.normal(0, sigma, clean.shape)), 0, 255)
    out, basic, groups = _denoise_keep(noisy, sigma)
    H, W = noisy.shape
    D = obm3d.dct8()
    thr = obm3d.LAMBDA_3D * sigma
    # stage 1
    ref1 = obm3d.stage1(noisy, sigma)
    explained1 = np.zeros((H, W), bool)
    for ry in obm3d.ref_positions(H):
        for rx in obm3d.ref_positions(W):
            pos = obm3d.match(noisy, ry, rx, obm3d.TAU_HT, obm3d.N2_HT)
            spec = obm3d.transform3d(np.stack([noisy[y:y + 8, x:x + 8] for y, x in pos]), D)
            if np.any(np.abs(np.abs(spec) - thr) <= EPS_C):
                _cover(explained1, pos)
    diff1 = np.abs(basic - ref1) > 1e-3
    print(f"stage 1: {int(diff1.sum())} pixels differ, {int(explained1.sum())} near a threshold tie")
    assert not np.any(diff1 & ~explained1), np.argwhere(diff1 & ~explained1)[:5]
    # stage 2, on the GPU's stage-1 estimate
    ref2 = obm3d.stage2(noisy, basic, sigma)
    explained2 = np.zeros((H, W), bool)
    n_refs = n_diff_groups = n_ambiguous = 0
    r = 0
    for ry in obm3d.ref_positions(H):
        for rx in obm3d.ref_positions(W):
            want = obm3d.match(basic, ry, rx, obm3d.TAU_WIE, obm3d.N2_WIE)
            amb = _ambiguous_match(basic, ry, rx, obm3d.TAU_WIE, obm3d.N2_WIE)
            n_refs += 1
            n_ambiguous += amb
            if groups[r] != want:
                n_diff_groups += 1
                assert amb, ((ry, rx), groups[r][:6], want[:6])
            if amb:
                _cover(explained2, want)
                _cover(explained2, groups[r])
            r += 1
    diff2 = np.abs(out - ref2) > 1e-3
    print(f"stage 2: {n_diff_groups} of {n_refs} groups differ ({n_ambiguous} ambiguous), "
          f"{int(diff2.sum())} pixels differ")
    assert not np.any(diff2 & ~explained2), np.argwhere(diff2 & ~explained2)[:5]
    assert np.mean(diff2) < 0.02
