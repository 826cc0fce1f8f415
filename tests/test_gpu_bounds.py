"""GPU parity of the full-sensing bounds THI / THB (Section IV) and of the
per-image correlation rho of Table 2, against the FP64 oracle.

Bars: kept counts per block bit-exact (both sides decide on the same float64
coefficients, computed in the same order); decoded pixels within 1e-3 of the
oracle's decoding of the kept coefficients rounded to float32 (the kernel's
contract: float32 transform of the kept set), and within 5e-3 of the exact
float64 decoding; rho within 1e-9.
"""
import numpy as np
import pytest

import synth
from oracle import abcs as orc
from oracle import bounds as ob

from gpu_util import pack_images, device

pytestmark = pytest.mark.gpu

PX_TOL = 1e-3
PX_TOL_F64 = 5e-3


class BoundRun:
    def __init__(self, px_host, entries):
        import torch
        import paper_2001_09632_amd as g
        dev = device()
        self.g = g
        self.plan = g.Plan(entries)
        self.px = torch.from_numpy(px_host).to(dev)
        nb, npx = self.plan.blocks, self.plan.pixels
        self.ws = torch.empty(g.threshold_workspace_bytes(self.plan), dtype=torch.uint8, device=dev)
        self.m = {r: torch.full((nb,), -7, dtype=torch.int32, device=dev) for r in ("thi", "thb")}
        self.out = {r: torch.full((max(1, npx),), float("nan"), dtype=torch.float32, device=dev)
                    for r in ("thi", "thb")}

    def run(self, rules=("thi", "thb"), decode=True):
        import torch
        for r in rules:
            self.g.threshold(self.plan, self.px, self.m[r], self.out[r] if decode else None, rule=r,
                             workspace=self.ws)
        torch.cuda.synchronize()
        self.h_m = {r: self.m[r].cpu().numpy() for r in rules}
        self.h_out = {r: self.out[r].cpu().numpy() for r in rules}
        return self

    def image(self, rule, i):
        d = self.plan.images[i]
        B = d["block"]
        hc, wc = d["cropped_height"], d["cropped_width"]
        b0, nb = d["block_offset"], (hc // B) * (wc // B)
        o0 = d["out_offset"]
        return self.h_m[rule][b0:b0 + nb], self.h_out[rule][o0:o0 + hc * wc].reshape(hc, wc)


def _decode32(img, B, keep):
    coefs = ob.coefficients(img, B)
    return ob._decode(coefs.astype(np.float32).astype(np.float64), keep, img, B)


def _check(run, j, img, B, cr, decode=True):
    m_ref, keep, rec = ob.thi(img, B, cr)
    m, out = run.image("thi", j)
    assert np.array_equal(m, m_ref), f"THI counts (entry {j}, B {B}, C_R {cr})"
    if decode:
        e32 = np.max(np.abs(out - _decode32(img, B, keep)))
        e64 = np.max(np.abs(out - rec))
        assert e32 < PX_TOL and e64 < PX_TOL_F64, f"THI pixels {e32} / {e64} (entry {j}, B {B}, C_R {cr})"
    keep_b, rec_b = ob.thb(img, B, cr)
    M, nB = ob.total_measurements(img, B, cr)
    m, out = run.image("thb", j)
    assert np.all(m == M // nB), f"THB counts (entry {j})"
    if decode:
        e32 = np.max(np.abs(out - _decode32(img, B, keep_b)))
        e64 = np.max(np.abs(out - rec_b))
        assert e32 < PX_TOL and e64 < PX_TOL_F64, f"THB pixels {e32} / {e64} (entry {j}, B {B}, C_R {cr})"


@pytest.mark.parametrize("B,sizes", [(16, [(64, 80), (131, 77), (256, 256), (16, 16)]),
                                     (8, [(72, 40), (131, 77), (8, 8)]),
                                     (32, [(96, 160), (200, 71), (32, 32)])])
def test_bounds_subrates_ragged(B, sizes):
    imgs = [synth.synth_image(900 + 5 * i + B, h, w) for i, (h, w) in enumerate(sizes)]
    px, d = pack_images(imgs, pitch_pad=4)
    entries, cases = [], []
    for i, img in enumerate(imgs):
        for cr in (0.01, 0.05, 0.1, 0.3, 0.5, 1.0):
            hc, wc = img.shape[0] // B * B, img.shape[1] // B * B
            if int(np.floor(cr * (hc * wc))) == 0:
                continue
            entries.append(dict(d[i], block=B, subrate=cr, method="zz"))
            cases.append((i, cr))
    run = BoundRun(px, entries).run()
    for j, (i, cr) in enumerate(cases):
        _check(run, j, imgs[i], B, cr)


def test_bounds_mixed_block_sizes_and_methods():
    imgs = [synth.synth_image(950 + i, 96 + 16 * i, 128) for i in range(3)]
    px, d = pack_images(imgs)
    entries = [dict(d[0], block=8, subrate=0.2, method="dd"), dict(d[1], block=16, subrate=0.15, method="bbv"),
               dict(d[2], block=32, subrate=0.3, method="zz"), dict(d[1], block=16, subrate=0.4, method="dd")]
    cases = [(0, 8, 0.2), (1, 16, 0.15), (2, 32, 0.3), (1, 16, 0.4)]
    run = BoundRun(px, entries).run()
    for j, (i, B, cr) in enumerate(cases):
        _check(run, j, imgs[i], B, cr)


def test_thi_ties_across_blocks():
    """Every block holds the same pixels, so every magnitude occurs once per
    block and the M-th largest is shared by all blocks: the lower blocks take
    the ties."""
    rng = np.random.default_rng(5)
    tile = rng.integers(0, 256, size=(16, 16), dtype=np.uint8)
    img = np.tile(tile, (4, 5))
    flat = np.full((48, 48), 77, np.uint8)
    px, d = pack_images([img, flat])
    crs = (0.1, 0.2337, 0.5)
    entries = [dict(d[0], block=16, subrate=cr, method="zz") for cr in crs]
    entries += [dict(d[1], block=16, subrate=cr, method="zz") for cr in crs]
    run = BoundRun(px, entries).run()
    for j, cr in enumerate(crs):
        _check(run, j, img, 16, cr)
        m, _ = run.image("thi", j)
        assert m.max() - m.min() <= 1 and np.all(np.diff(m) <= 0), "ties must favour the lower blocks"
        _check(run, len(crs) + j, flat, 16, cr)


@pytest.mark.parametrize("size", [256, 64])
def test_budget_correlation_matches_oracle(size):
    """rho and its p-value per image (64 x 64: 16 blocks, p of order 1e-3
    .. 1; 256 x 256: 256 blocks, p down to ~1e-100)."""
    import torch
    import paper_2001_09632_amd as g
    from gpu_util import Run
    imgs = [synth.synth_image(970 + i + size, size, size) for i in range(3)]
    px, d = pack_images(imgs)
    crs = (0.1, 0.3, 0.5)
    entries, cases = [], []
    for i in range(3):
        for cr in crs:
            for meth in ("bbv", "dd", "zz"):
                try:
                    orc.budget_scalars(size, size, 16, cr, orc.METHOD_NAMES[meth])
                except orc.DomainError:
                    continue
                entries.append(dict(d[i], block=16, subrate=cr, method=meth))
                cases.append((i, cr, meth))
    est = Run(px, entries).budget()
    bnd = BoundRun(px, entries)
    bnd.run(rules=("thi",), decode=False)
    rho = torch.full((len(entries),), -7.0, dtype=torch.float64, device=device())
    pv = torch.full((len(entries),), -7.0, dtype=torch.float64, device=device())
    g.budget_correlation(bnd.plan, bnd.m["thi"], est.k, rho, pv)
    est.fetch()
    rho_h, p_h = rho.cpu().numpy(), pv.cpu().numpy()
    for j, (i, cr, meth) in enumerate(cases):
        m_ref, _, _ = ob.thi(imgs[i], 16, cr)
        k_ref, _ = orc.budget(imgs[i], 16, cr, orc.METHOD_NAMES[meth])
        want = ob.pearson(m_ref, k_ref)
        if np.isnan(want):
            assert np.isnan(rho_h[j]) and np.isnan(p_h[j]), f"constant budget must give NaN ({meth})"
            continue
        assert abs(rho_h[j] - want) < 1e-9, f"rho {rho_h[j]} vs {want} ({meth}, C_R {cr})"
        p_ref = ob.pearson_p(want, m_ref.size)
        assert abs(p_h[j] - p_ref) <= 1e-9 * p_ref + 1e-300, f"p {p_h[j]} vs {p_ref} ({meth}, C_R {cr})"


def test_bounds_full_size_512():
    """512 x 512 images at B = 16 in one plan (the launch shape of the timed
    bound): every count exact, decoded pixels on a sample of rows."""
    imgs = [synth.synth_image(990 + i, 512, 512) for i in range(4)]
    px, d = pack_images(imgs)
    crs = (0.1, 0.25, 0.4, 0.5)
    entries = [dict(d[i], block=16, subrate=crs[i], method="dd") for i in range(4)]
    run = BoundRun(px, entries).run()
    rows = np.random.default_rng(1).choice(512, size=24, replace=False)
    for j in range(4):
        img, cr = imgs[j], crs[j]
        m_ref, keep, rec = ob.thi(img, 16, cr)
        m, out = run.image("thi", j)
        assert np.array_equal(m, m_ref)
        assert np.max(np.abs(out[rows] - _decode32(img, 16, keep)[rows])) < PX_TOL
        keep_b, _ = ob.thb(img, 16, cr)
        m, out = run.image("thb", j)
        assert np.max(np.abs(out[rows] - _decode32(img, 16, keep_b)[rows])) < PX_TOL


def test_threshold_errors():
    import torch
    import paper_2001_09632_amd as g
    img = synth.synth_image(3, 32, 32)
    px, d = pack_images([img])
    run = BoundRun(px, [dict(d[0], block=16, subrate=0.2, method="zz")])
    with pytest.raises(g.AbcsError, match="EINVAL"):
        g.threshold(run.plan, run.px, run.m["thi"], rule=3, workspace=run.ws)
    small = torch.empty(16, dtype=torch.uint8, device=device())
    with pytest.raises(g.AbcsError, match="ENOSPACE"):
        g.threshold(run.plan, run.px, run.m["thi"], rule="thi", workspace=small)


def test_thi_all_zero_image_ties_everywhere():
    """Every coefficient of a black image is 0: all magnitudes tie, so THI
    fills blocks in raster order, each in zigzag order."""
    img = np.zeros((48, 64), np.uint8)
    px, d = pack_images([img])
    crs = (0.1, 0.5, 0.9)
    run = BoundRun(px, [dict(d[0], block=16, subrate=cr, method="zz") for cr in crs]).run()
    for j, cr in enumerate(crs):
        _check(run, j, img, 16, cr)
        m, out = run.image("thi", j)
        M = int(np.floor(cr * 48 * 64))
        want = np.minimum(np.maximum(M - 256 * np.arange(12), 0), 256)
        assert np.array_equal(m, want)
        assert np.all(out == 0.0)
