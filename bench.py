#!/usr/bin/env python3
"""Throughput of adaptive block compressive sensing on one MI355X.

Workload (one step): a batch of 64 synthetic 512x512 uint8 greyscale images
(seeds 1000..1063), B = 16, both budget estimators (AL-DCT-BBV and
AL-DCT-DD) at subrates 0.1, 0.2, 0.3, 0.4, 0.5 - 640 image encodings in one
plan - run through phase-1 statistics + budget apportionment (abcs_budget)
and phase-2 sensing with the masked inverse 2D-DCT decoder in one pass
(abcs_sense_decode), float32: the two launches of abcs_encode.  Inputs are
resident in HBM before timing starts.

Prints one JSON line: Mpixel/s over the whole step, the roofline of the
dominant kernel (HIP events on the launch stream) and of the whole step,
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SETTLE_S = 0.5             # untimed work before the warmup steps (clocks leave idle)
BF16_PEAK_TFLOPS = 2500.0   # dense bf16 matrix-core peak of MI355X
SEEDS = list(range(1000, 1064))
SUBRATES = (0.1, 0.2, 0.3, 0.4, 0.5)
METHODS = ("bbv", "dd")
H = W = 512
B = 16


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_images():
    import numpy as np
    import synth
    return np.stack([synth.synth_image(s, H, W) for s in SEEDS])


def entries():
    out = []
    for m in METHODS:
        for cr in SUBRATES:
            for i in range(len(SEEDS)):
                out.append(dict(height=H, width=W, row_pitch=W, block=B, subrate=cr, method=m,
                                pixel_offset=i * H * W))
    return out


def algorithmic_bytes(plan, kind):
    """Bytes each launch must move at least, from the plan's sizes.

    reconstruct: read y (4 B per coefficient), k (4 B/block), offsets
                 (8 B/block); write the decoded image (4 B/pixel).
    sense:       read the pixels (1 B/pixel), k, offsets; write y.
    """
    if kind == "reconstruct":
        return 4 * plan.meas + 12 * plan.blocks + 4 * plan.pixels
    if kind == "sense":
        return plan.pixels + 12 * plan.blocks + 4 * plan.meas
    if kind == "sense_decode":
        return plan.pixels + 12 * plan.blocks + 4 * plan.meas + 4 * plan.pixels
    raise ValueError(kind)


def oracle_decodes(images, plan, k_all, n_images=8):
    """The float64 oracle's decoding of its own measurements for the first
    n_images at every (estimator, subrate) pair: {plan image index: image}.
    The budgets are the GPU's, which equal the oracle's bit for bit (checked
    here as well)."""
    from oracle import abcs as orc
    out = {}
    for j, d in enumerate(plan.images):
        i = j % len(SEEDS)
        if i >= n_images:
            continue
        m = METHODS[j // (len(SEEDS) * len(SUBRATES))]
        cr = SUBRATES[(j // len(SEEDS)) % len(SUBRATES)]
        k, _ = orc.budget(images[i], B, cr, orc.METHOD_NAMES[m])
        b0 = d["block_offset"]
        assert (k_all[b0:b0 + k.size] == k).all(), "budget differs from the oracle"
        out[j] = orc.reconstruct(orc.sense(images[i], B, k), B, k, H, W)
    return out


def precision_errors(plan, out_host, sample, images):
    """Largest |pixel - oracle pixel| and mean |dPSNR| (clean image as
    reference) over the sampled encodings."""
    import numpy as np
    from oracle import metrics
    mx, dp = 0.0, []
    for j, ref in sample.items():
        d = plan.images[j]
        got = out_host[d["out_offset"]:d["out_offset"] + H * W].reshape(H, W).astype(np.float64)
        mx = max(mx, float(np.max(np.abs(got - ref))))
        clean = images[j % len(SEEDS)].astype(np.float64)
        dp.append(abs(metrics.psnr(got, clean) - metrics.psnr(ref, clean)))
    return {"max_abs_dpx_vs_oracle": round(mx, 6), "mean_abs_dpsnr_vs_oracle_db": round(float(np.mean(dp)), 6),
            "max_abs_dpsnr_vs_oracle_db": round(float(np.max(dp)), 6), "sampled_encodings": len(sample)}


# HBM traffic of a kernel on this workload: rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads for
# a plain device copy of 1 GiB (`bench.py --copy-probe 1024`).  A reading holds
# only for the kernel it was taken on, so it is keyed by the SHA-256 of the
# files that define the kernel and of the compiler flags (source_key); after
# any change the figure is null until the counters are taken again.
COPY_KIB = 1048576.0
TRAFFIC = {
    "sense_decode": dict(
        sources=("csrc/common.hpp", "csrc/transform16.hpp", "csrc/sense_kernels.hpp"),
        sha256="8512e41aa27704bb57562ee7ecdbff1390b6b28cd6847511bf57bacc0677b3db",
        fetch_kib=58694.46, write_kib=840648.46,
        copy_fetch_kib=524301.21, copy_write_kib=1048576.0),
}


# Float32 arithmetic of one BM3D call on the IDA batch at sigma 25, counted
# with rocprofv3 (SQ_INSTS_VALU_ADD/MUL/FMA/TRANS_F32, 64 lanes per wave
# instruction, FMA = 2 flops; an upper bound, masked lanes count); keyed like
# TRAFFIC by the sources that define the kernels.
BM3D_FP32 = dict(sources=("csrc/bm3d_kernels.hpp",),
                 sha256="0432df4b373cc789e3ad2c121ec95c902704d78ff5d959167eab017ca4c7ce96", flop_per_call=5.41e11)
FP32_PEAK_TFLOPS = 157.3


def source_key(sources):
    """SHA-256 of the code of the files that define a kernel (comments aside)
    and of the compiler flags."""
    import hashlib
    from paper_2001_09632_amd import build
    h = hashlib.sha256(" ".join(build.FLAGS).encode())
    for f in sources:
        with open(os.path.join(ROOT, "paper_2001_09632_amd", f), "rb") as fh:
            h.update(build.code_text(fh.read()))
    return h.hexdigest()


def counted_bm3d_flop():
    return BM3D_FP32["flop_per_call"] if source_key(BM3D_FP32["sources"]) == BM3D_FP32["sha256"] else None


def measured_traffic(kind):
    """HBM bytes per launch from the counter readings above, or None."""
    t = TRAFFIC.get(kind)
    if t is None or source_key(t["sources"]) != t["sha256"]:
        return None
    fetch = t["fetch_kib"] * COPY_KIB / t["copy_fetch_kib"]
    write = t["write_kib"] * COPY_KIB / t["copy_write_kib"]
    return int(round((fetch + write) * 1024))


IDA_SEEDS = list(range(2000, 2032))
IDA_SIZES = [256] * 16 + [512] * 16
IDA_ITERS = 30


def ida_workload():
    """16 x 256^2 + 16 x 512^2 synthetic images, C_R ~ U(0.1, 0.3) drawn from
    stream seed 3, AL-DCT-DD on even and AL-DCT-BBV on odd images, B = 16."""
    import numpy as np
    import synth
    crs = np.random.default_rng(3).uniform(0.1, 0.3, size=len(IDA_SEEDS))
    imgs = [synth.synth_image(s, n, n) for s, n in zip(IDA_SEEDS, IDA_SIZES)]
    methods = ["dd" if i % 2 == 0 else "bbv" for i in range(len(imgs))]
    return imgs, crs, methods


def judge_section(dev, plan, y, k, off, imgs, prm, capture=(1, 3, 5, 10, 20, 29)):
    """The plain denoiser as judge of the learned one: pairs (v^t, sigma^t)
    captured from the plain (BM3D) loop on the IDA batch (images never used
    in training) at the iterations in `capture`, each denoised by the CNN
    (with its fallback) and by BM3D; mean squared error against the clean
    image, for the pairs whose sigma lies in the network's accepted range and
    for all pairs."""
    import numpy as np
    import torch
    import paper_2001_09632_amd as g
    n = plan.n
    ws = torch.empty(g.ida_workspace_bytes(plan, "bm3d"), dtype=torch.uint8, device=dev)
    wc = torch.empty(g.denoise_workspace_bytes(plan, "cnn"), dtype=torch.uint8, device=dev)
    wb = torch.empty(g.denoise_workspace_bytes(plan, "bm3d"), dtype=torch.uint8, device=dev)
    x = torch.zeros(plan.pixels, dtype=torch.float32, device=dev)
    v = torch.empty_like(x)
    oc, ob = torch.empty_like(x), torch.empty_like(x)
    sig = torch.empty(n, dtype=torch.float32, device=dev)
    lo, hi = float(prm[-2]), float(prm[-1])
    mse_c, mse_b, inr = [], [], []
    for t in range(max(capture) + 1):
        g.ida_iterate(plan, y, k, off, x, t, t + 1, 2.0, "bm3d", sigma_trace=sig, v_last=v, workspace=ws)
        if t not in capture:
            continue
        g.denoise(plan, v, sig, oc, "cnn", params=prm, workspace=wc)
        g.denoise(plan, v, sig, ob, "bm3d", workspace=wb)
        torch.cuda.synchronize()
        hc, hb, hs = oc.cpu().numpy(), ob.cpu().numpy(), sig.cpu().numpy()
        for i, im in enumerate(imgs):
            d = plan.images[i]
            ref = im.astype(np.float64).reshape(-1)
            a = hc[d["out_offset"]:d["out_offset"] + im.size].astype(np.float64)
            b = hb[d["out_offset"]:d["out_offset"] + im.size].astype(np.float64)
            mse_c.append(float(np.mean((a - ref) ** 2)))
            mse_b.append(float(np.mean((b - ref) ** 2)))
            inr.append(lo <= float(hs[i]) <= hi)
    mse_c, mse_b, inr = np.array(mse_c), np.array(mse_b), np.array(inr)
    return {"pairs": int(mse_c.size), "iterations": list(capture),
            "accepted_sigma_range": [lo, hi if np.isfinite(hi) else "inf"],
            "in_range": {"pairs": int(inr.sum()), "cnn_mse": round(float(mse_c[inr].mean()), 3),
                         "bm3d_mse": round(float(mse_b[inr].mean()), 3),
                         "cnn_better_fraction": round(float(np.mean(mse_c[inr] < mse_b[inr])), 3)},
            "all": {"cnn_mse": round(float(mse_c.mean()), 3), "bm3d_mse": round(float(mse_b.mean()), 3)}}


def ida_oracle_sample(dev, imgs, prm, iters=5, size=64):
    """Config 3 against the FP64 oracle on a bounded sample: the top-left
    size x size crops of the IDA batch's first two images (DD at C_R 0.2,
    BBV at 0.25), `iters` IDA iterations with BM3D and with the CNN on the GPU
    and in the oracle (the oracle's CNN rounds weights and hidden activations
    to bfloat16, as the network's arithmetic is defined, and falls back to
    BM3D outside the trained sigma range); PSNR against the clean crop."""
    import numpy as np
    import torch
    import paper_2001_09632_amd as g
    from oracle import bm3d as obm3d, cnn as ocnn, ida as oida, metrics
    from paper_2001_09632_amd.train import encode_batch
    crops = [np.ascontiguousarray(im[:size, :size]) for im in imgs[:2]]
    plan, y, k, off = encode_batch(dev, crops, [0.2, 0.25], ["dd", "bbv"])
    pr = prm.cpu().numpy().astype(np.float64)
    blob, lo, hi = pr[:-2], pr[-2], pr[-1]

    def bf16(a):
        u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        return u.astype(np.uint32).view(np.float32).astype(np.float64)

    layers = [(bf16(w), b) for w, b in ocnn.unpack(blob)]

    def cnn_oracle(vv, sg):
        if not (lo <= sg <= hi):
            return obm3d.bm3d(vv, sg)
        a = ocnn.network_input(vv[None], [sg])
        for i, (w, b) in enumerate(layers):
            a = ocnn.conv3x3(a, w, b)
            if i < len(layers) - 1:
                a = bf16(np.maximum(a, 0.0))
        return vv - 255.0 * a[0, ..., 0]

    yh, kh = y.cpu().numpy(), k.cpu().numpy()
    out = {"sample": f"{len(crops)} crops of {size}x{size}, {iters} iterations, D_F = 2"}
    for den, params, oden in (("bm3d", None, obm3d.bm3d), ("cnn", prm, cnn_oracle)):
        ws = torch.empty(g.ida_workspace_bytes(plan, den), dtype=torch.uint8, device=dev)
        x = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
        g.ida_refine(plan, y, k, off, x, iters, 2.0, den, params=params, workspace=ws)
        torch.cuda.synchronize()
        xh = x.cpu().numpy().astype(np.float64)
        pg, po = [], []
        for i, c in enumerate(crops):
            d = plan.images[i]
            nb = (size // 16) ** 2
            yi = yh[d["meas_offset"]:d["meas_offset"] + d["n_meas"]].astype(np.float64)
            xo, _ = oida.ida(yi, kh[d["block_offset"]:d["block_offset"] + nb], 16, size, size, iters, 2.0,
                             denoiser=oden)
            pg.append(metrics.psnr(xh[d["out_offset"]:d["out_offset"] + c.size].reshape(c.shape), c.astype(float)))
            po.append(metrics.psnr(xo, c.astype(float)))
        out[den] = {"psnr_gpu": round(float(np.mean(pg)), 4), "psnr_oracle": round(float(np.mean(po)), 4),
                    "max_abs_dpsnr_db": round(float(np.max(np.abs(np.array(pg) - np.array(po)))), 4)}
    return out


def ida_section(dev, weights_path):
    """Plain IDA (BM3D, 30 iterations, D_F = 2) against learned IDA (CNN) on
    one mixed batch: images/s and PSNR/SSIM against the ground truth; the
    learned loop runs the fewest of 5, 10, ..., 30 iterations that reaches the
    plain loop's PSNR minus 0.1 dB."""
    import numpy as np
    import torch
    import paper_2001_09632_amd as g
    from paper_2001_09632_amd import quality
    from paper_2001_09632_amd.train import encode_batch, load_params
    imgs, crs, methods = ida_workload()
    plan, y, k, off = encode_batch(dev, imgs, crs, methods)
    n = len(imgs)

    def scores(x):
        h = x.cpu().numpy()
        ps, ss = [], []
        for i, im in enumerate(imgs):
            d = plan.images[i]
            est = h[d["out_offset"]:d["out_offset"] + im.size].reshape(im.shape)
            ps.append(quality.psnr(est, im))
            ss.append(quality.ssim(est, im))
        return float(np.mean(ps)), float(np.mean(ss))

    def timed(iters, den, params=None):
        # the whole loop is recorded once as a HIP graph; the timed region is
        # one replay (after one untimed replay)
        ws = torch.empty(g.ida_workspace_bytes(plan, den), dtype=torch.uint8, device=dev)
        x = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
        graph = g.IdaGraph(plan, y, k, off, x, iters, 2.0, den, params=params, workspace=ws)
        graph.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.launch()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        graph.close()
        return dt, x

    io = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    g.reconstruct(plan, y, k, off, io)
    io_p, io_s = scores(io)
    tp, xp = timed(IDA_ITERS, "bm3d")
    pp, sp = scores(xp)
    rec = {"workload": "16x256^2 + 16x512^2 synthetic images, C_R ~ U(0.1,0.3), B=16, D_F=2",
           "images": n, "io": {"psnr": round(io_p, 3), "ssim": round(io_s, 4)},
           "plain": {"denoiser": "bm3d", "iters": IDA_ITERS, "images_per_s": round(n / tp, 2),
                     "ms_per_batch": round(tp * 1e3, 2), "psnr": round(pp, 3), "ssim": round(sp, 4)}}
    if not os.path.exists(weights_path):
        rec["learned"] = None
        rec["note"] = f"no CNN weights at {weights_path}"
        return rec
    prm = torch.from_numpy(load_params(weights_path)).to(dev)
    trail, trail_t = {}, {}
    chosen = None
    for it in (5, 10, 15, 20, 25, 30):
        tl, xl = timed(it, "cnn", prm)
        pl, sl = scores(xl)
        trail[it] = round(pl, 3)
        trail_t[it] = tl
        if chosen is None and pl >= pp - 0.1:
            chosen = (it, tl, pl, sl)
    matched = chosen is not None
    if not matched:
        tl, xl = timed(IDA_ITERS, "cnn", prm)
        pl, sl = scores(xl)
        chosen = (IDA_ITERS, tl, pl, sl)
    it, tl, pl, sl = chosen
    rec["learned"] = {"denoiser": "cnn", "iters": it, "images_per_s": round(n / tl, 2),
                      "ms_per_batch": round(tl * 1e3, 2), "psnr": round(pl, 3), "ssim": round(sl, 4),
                      "psnr_by_iters": trail}
    rec["matched_psnr"] = matched
    rec["learned_over_plain_images_per_s"] = round(tp / tl, 2)
    # both loops at the plain loop's iteration count
    rec["learned_at_plain_iters"] = {"iters": IDA_ITERS, "images_per_s": round(n / trail_t[IDA_ITERS], 2),
                                     "psnr": trail[IDA_ITERS],
                                     "over_plain_images_per_s": round(tp / trail_t[IDA_ITERS], 2)}

    rec["judge"] = judge_section(dev, plan, y, k, off, imgs, prm)
    rec["vs_oracle"] = ida_oracle_sample(dev, imgs, prm)

    # Roofline of the learned denoisers alone (one abcs_denoise call on the
    # batch, HIP events on the launch stream): algorithmic flops of the
    # convolutions (2 x 9 x C_in x C_out per pixel and layer) against the
    # dense bf16 matrix-core peak.
    def denoise_ms(den, params, reps=5):
        ws = torch.empty(g.denoise_workspace_bytes(plan, den), dtype=torch.uint8, device=dev)
        sig = torch.full((n,), 25.0, dtype=torch.float32, device=dev)
        o = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
        g.denoise(plan, io, sig, o, den, params=params, workspace=ws)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            g.denoise(plan, io, sig, o, den, params=params, workspace=ws)
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    def conv_roofline(ms, n_mid):
        flop = plan.pixels * 2 * 9 * (2 * 64 + n_mid * 64 * 64 + 64)
        ach = flop / (ms * 1e-3) / 1e12
        return {"ms_per_call": round(ms, 3), "bound": "mfma", "achieved": round(ach, 1), "peak": BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / BF16_PEAK_TFLOPS, 4), "algorithmic_flop": int(flop)}

    bm3d_ms = denoise_ms("bm3d", None, reps=2)
    bm3d_flop = counted_bm3d_flop()
    rec["denoiser_roofline"] = {"cnn": conv_roofline(denoise_ms("cnn", prm), 6),
                                "bm3d_ms_per_call": round(bm3d_ms, 3),
                                "bm3d": None if bm3d_flop is None else {
                                    "ms_per_call": round(bm3d_ms, 3), "bound": "valu issue",
                                    "counted_fp32_flop": bm3d_flop,
                                    "achieved": round(bm3d_flop / (bm3d_ms * 1e-3) / 1e12, 1),
                                    "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                    "frac": round(bm3d_flop / (bm3d_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4)}}

    # DnCNN-17 with batch normalisation (the paper's network, trained here by
    # the library's kernels): the same matched-PSNR rule.
    dn_path = os.path.join(os.path.dirname(weights_path), "ida_dncnn.npy")
    if os.path.exists(dn_path):
        dprm = torch.from_numpy(load_params(dn_path, arch="dncnn")).to(dev)
        dtrail, dtrail_t, dchosen = {}, {}, None
        for itd in (5, 10, 15, 20, 25, 30):
            td, xd = timed(itd, "dncnn", dprm)
            pd_, sd = scores(xd)
            dtrail[itd] = round(pd_, 3)
            dtrail_t[itd] = td
            if dchosen is None and pd_ >= pp - 0.1:
                dchosen = (itd, td, pd_, sd)
        if dchosen is None:
            td, xd = timed(IDA_ITERS, "dncnn", dprm)
            dchosen = (IDA_ITERS, td) + scores(xd)
        itd, td, pd_, sd = dchosen
        rec["dncnn"] = {"denoiser": "dncnn-17", "iters": itd, "images_per_s": round(n / td, 2),
                        "ms_per_batch": round(td * 1e3, 2), "psnr": round(pd_, 3), "ssim": round(sd, 4),
                        "psnr_by_iters": dtrail, "over_plain_images_per_s": round(tp / td, 2),
                        "at_plain_iters": {"iters": IDA_ITERS, "images_per_s": round(n / dtrail_t[IDA_ITERS], 2),
                                           "psnr": dtrail[IDA_ITERS],
                                           "over_plain_images_per_s": round(tp / dtrail_t[IDA_ITERS], 2)}}
        rec["denoiser_roofline"]["dncnn"] = conv_roofline(denoise_ms("dncnn", dprm), 15)

    # The loop variants of Section VI with the learned denoiser at the chosen
    # iteration count: IDA against D-AMP (eq 24) and DAMP-D (eq 27, D_F = 2),
    # and IDA's PSNR as a function of D_F (the sweep of Fig 8).
    probe = torch.from_numpy(np.random.default_rng(11).standard_normal(plan.pixels).astype(np.float32)).to(dev)
    wsa = torch.empty(g.amp_workspace_bytes(plan, "cnn"), dtype=torch.uint8, device=dev)
    xa = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    variants = {}
    for name, alg in (("d-amp", "damp"), ("damp-d", "damp-d")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.amp_refine(plan, y, k, off, xa, it, probe, damping=2.0, algorithm=alg, denoiser="cnn", params=prm,
                     workspace=wsa)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pa, sa = scores(xa)
        variants[name] = {"iters": it, "psnr": round(pa, 3), "ssim": round(sa, 4), "ms_per_batch": round(dt * 1e3, 2)}
    variants["ida"] = {"iters": it, "psnr": round(pl, 3), "ssim": round(sl, 4), "ms_per_batch": round(tl * 1e3, 2)}
    rec["loop_variants"] = variants
    wsi = torch.empty(g.ida_workspace_bytes(plan, "cnn"), dtype=torch.uint8, device=dev)
    sweep = {}
    for df in (1.0, 1.25, 1.5, 2.0, 3.0, 4.0):
        g.ida_refine(plan, y, k, off, xa, it, df, "cnn", params=prm, workspace=wsi)
        sweep[str(df)] = round(scores(xa)[0], 3)
    rec["ida_psnr_by_damping"] = sweep

    # The BBV images' phase-1 samples as extra measurements (Section V-A):
    # learned IDA on the BBV images with and without them as rows of A.
    px = torch.from_numpy(np.concatenate([im.reshape(-1) for im in imgs])).to(dev)
    bbv = torch.empty(max(1, plan.bbv_total), dtype=torch.float32, device=dev)
    g.bbv_samples(plan, px, bbv)
    sel = [i for i in range(n) if methods[i] == "bbv"]

    def psnr_sel(x):
        h = x.cpu().numpy()
        out = []
        for i in sel:
            d = plan.images[i]
            out.append(quality.psnr(h[d["out_offset"]:d["out_offset"] + imgs[i].size].reshape(imgs[i].shape), imgs[i]))
        return round(float(np.mean(out)), 3)

    g.ida_refine(plan, y, k, off, xa, it, 2.0, "cnn", params=prm, workspace=wsi)
    p_plain = psnr_sel(xa)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.ida_refine_bbv(plan, y, k, off, bbv, xa, it, 2.0, "cnn", params=prm, workspace=wsi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rec["bbv_rows"] = {"images": len(sel), "iters": it, "samples": int(plan.bbv_total),
                       "psnr_without": p_plain, "psnr_with": psnr_sel(xa), "ms_per_batch": round(dt * 1e3, 2)}
    return rec


STREAM_SIZES = [(256, 256), (512, 512), (768, 1024), (2048, 2048)]   # (H, W); 1024x768 read as W x H
STREAM_BUDGET_BYTES = 1 << 30   # device bytes of y, decoded images and per-block arrays admitted per batch


def single_image_section(dev, reps=200):
    """One 256x256 synthetic image (seed 0), B = 16, AL-DCT-BBV at C_R 0.25,
    float32: abcs_encode (budget, sensing and the decoder's image) per call,
    latency-bound at this size; budgets checked against the oracle and the
    decoded pixels against the oracle's decoding of its own float64
    measurements."""
    import numpy as np
    import torch
    import paper_2001_09632_amd as g
    import synth
    from oracle import abcs as orc
    img = synth.synth_image(0, 256, 256)
    px = torch.from_numpy(img.reshape(-1)).to(dev)
    plan = g.Plan([dict(height=256, width=256, row_pitch=256, block=16, subrate=0.25, method="bbv",
                        pixel_offset=0)])
    k = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    off = torch.empty(plan.blocks, dtype=torch.int64, device=dev)
    st = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    y = torch.empty(plan.meas, dtype=torch.float32, device=dev)
    out = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    for _ in range(10):
        g.encode(plan, px, k, off, st, y, out)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    for _ in range(reps):
        g.encode(plan, px, k, off, st, y, out)
    e[1].record()
    torch.cuda.synchronize()
    ms = e[0].elapsed_time(e[1]) / reps
    kk, _, yy = orc.encode(img, 16, 0.25, orc.BBV)
    ref = orc.reconstruct(yy, 16, kk, 256, 256)
    return {"workload": "one 256x256 synthetic image (seed 0), B=16, AL-DCT-BBV, C_R 0.25, float32, abcs_encode",
            "ms_per_image": round(ms, 4), "mpixel_per_s": round(65536 / ms / 1e3, 1),
            "budgets_equal_oracle": bool(np.array_equal(k.cpu().numpy(), kk)),
            "max_abs_dpx_vs_oracle": round(float(np.max(np.abs(out.cpu().numpy().reshape(256, 256) - ref))), 6)}


def stream_requests(n, seed=5):
    """n requests of the mixed stream: size uniform over STREAM_SIZES, B over
    {8, 16, 32}, C_R ~ U(0.05, 0.5), budget rule over {ZZ, BBV, DD}."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return [dict(size=int(rng.integers(0, 4)), block=int(rng.choice([8, 16, 32])),
                 subrate=float(rng.uniform(0.05, 0.5)), method=str(rng.choice(["zz", "bbv", "dd"])))
            for _ in range(n)]


def stream_precision_errors(dev, reqs, pool, offs, px, entry, n_sample=24):
    """Every precision mode on a sample of the stream's requests (the first
    n_sample of size at most 1024x768: all three block sizes, rules and a
    spread of C_R) in one plan: largest |pixel - oracle pixel| and mean /
    largest |dPSNR| (clean image as reference), the oracle decoding its own
    float64 measurements with the same budgets (the GPU's budgets equal the
    oracle's, checked here too)."""
    import numpy as np
    import torch
    import paper_2001_09632_amd as g
    from oracle import abcs as orc
    from oracle import metrics
    idx = [i for i, r in enumerate(reqs) if STREAM_SIZES[r["size"]][0] * STREAM_SIZES[r["size"]][1] <= 1024 * 768]
    idx = idx[:n_sample]
    plan = g.Plan([entry(reqs[i]) for i in idx], features=())
    k = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    off = torch.empty(plan.blocks, dtype=torch.int64, device=dev)
    st = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    y = torch.empty(plan.meas, dtype=torch.float32, device=dev)
    out = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    g.budget(plan, px, k, off, st)
    kh = k.cpu().numpy()
    refs = []
    for j, i in enumerate(idx):
        r, d = reqs[i], plan.images[j]
        img = pool[r["size"]]
        kk, _ = orc.budget(img, r["block"], r["subrate"], orc.METHOD_NAMES[r["method"]])
        assert np.array_equal(kh[d["block_offset"]:d["block_offset"] + kk.size], kk), "budget differs from the oracle"
        h, w = img.shape
        refs.append((orc.reconstruct(orc.sense(img, r["block"], kk), r["block"], kk, h, w), d))
    res = {"sample": f"{len(idx)} requests (B 8/16/32, ZZ/BBV/DD, sizes up to 1024x768)"}
    for mode in g.PRECISIONS:
        g.sense_decode(plan, px, k, off, y, out, precision=mode)
        oh = out.cpu().numpy()
        mx, dp = 0.0, []
        for (ref, d), i in zip(refs, idx):
            hc, wc = d["cropped_height"], d["cropped_width"]
            got = oh[d["out_offset"]:d["out_offset"] + hc * wc].reshape(hc, wc).astype(np.float64)
            clean = pool[reqs[i]["size"]][:hc, :wc].astype(np.float64)
            mx = max(mx, float(np.max(np.abs(got - ref))))
            dp.append(abs(metrics.psnr(got, clean) - metrics.psnr(ref, clean)))
        res[mode] = {"max_abs_dpx_vs_oracle": round(mx, 6), "mean_abs_dpsnr_db": round(float(np.mean(dp)), 6),
                     "max_abs_dpsnr_db": round(float(np.max(dp)), 6)}
    return res


def stream_section(dev, n_requests=1000, load=0.5):
    """The mixed request stream: every request is encoded (budget + sense) and
    decoded (masked inverse DCT) on the GPU with abcs_encode.  Requests are
    batched in arrival order while their y and decoded images fit
    STREAM_BUDGET_BYTES; one plan per batch (host work: timed apart from the
    GPU work in the saturated run, inside the latency in the stream).  Image content comes
    from a pool of one synthetic image per size held in device memory.  First
    all requests arrive at once (saturated Mpixel/s), then as a Poisson stream
    (seed 7) at `load` times the saturated pixel rate; latency = completion -
    arrival."""
    import numpy as np
    import torch
    import paper_2001_09632_amd as g
    import synth
    pool = [synth.synth_image(3000 + i, h, w) for i, (h, w) in enumerate(STREAM_SIZES)]
    offs, o = [], 0
    for im in pool:
        offs.append(o)
        o += im.size
    px = torch.from_numpy(np.concatenate([im.reshape(-1) for im in pool])).to(dev)
    reqs = stream_requests(n_requests)

    def entry(r):
        h, w = STREAM_SIZES[r["size"]]
        return dict(height=h, width=w, row_pitch=w, block=r["block"], subrate=r["subrate"], method=r["method"],
                    pixel_offset=offs[r["size"]])

    # admission control: requests join the open batch in arrival order while
    # the batch's outputs (y, decoded images, per-block arrays) fit the budget
    admission = g.Admission(STREAM_BUDGET_BYTES)

    def batches(order):
        order = list(order)
        return [[order[j] for j in b] for b in admission.batches([entry(reqs[i]) for i in order])]

    max_blocks = max(sum((STREAM_SIZES[reqs[i]["size"]][0] // reqs[i]["block"]) *
                         (STREAM_SIZES[reqs[i]["size"]][1] // reqs[i]["block"]) for i in b)
                     for b in batches(range(n_requests)))
    kb = torch.empty(max_blocks, dtype=torch.int32, device=dev)
    ob = torch.empty(max_blocks, dtype=torch.int64, device=dev)
    sb = torch.empty(max_blocks, dtype=torch.int32, device=dev)
    yb = torch.empty(STREAM_BUDGET_BYTES // 4, dtype=torch.float32, device=dev)
    xb = torch.empty(STREAM_BUDGET_BYTES // 4, dtype=torch.float32, device=dev)

    plan_s = []

    def make_plan(idx):
        t = time.perf_counter()
        plan = g.Plan([entry(reqs[i]) for i in idx], features=())
        plan_s.append(time.perf_counter() - t)
        return plan

    def run_plan(plan):
        g.encode(plan, px, kb, ob, sb, yb, xb)
        torch.cuda.synchronize()
        return plan.pixels

    run_plan(make_plan(list(range(min(8, n_requests)))))          # warm up
    # saturated: every request at once; the batches' plans are made first
    # (host work, timed on its own), then the GPU runs them back to back
    plan_s.clear()
    plans = [make_plan(b) for b in batches(range(n_requests))]
    plan_total_s = sum(plan_s)
    t0 = time.perf_counter()
    total_px = 0
    for plan in plans:
        total_px += run_plan(plan)
    sat_s = time.perf_counter() - t0
    sat_rate = total_px / sat_s
    del plans

    def run_batch(idx):
        return run_plan(make_plan(idx))

    # Poisson arrivals at `load` of the saturated end-to-end pixel rate (the
    # stream plans each batch when it forms, so planning is part of the
    # service time)
    rng = np.random.default_rng(7)
    mean_px = total_px / n_requests
    e2e_rate = total_px / (sat_s + plan_total_s)
    gaps = rng.exponential(mean_px / (load * e2e_rate), size=n_requests)
    arrive = np.cumsum(gaps)
    done = np.zeros(n_requests)
    nxt = 0
    t0 = time.perf_counter()
    while nxt < n_requests:
        now = time.perf_counter() - t0
        if arrive[nxt] > now:
            time.sleep(arrive[nxt] - now)
            now = time.perf_counter() - t0
        ready = [i for i in range(nxt, n_requests) if arrive[i] <= now]
        batch = [ready[j] for j in admission.first_batch([entry(reqs[i]) for i in ready])]
        run_batch(batch)
        done[batch] = time.perf_counter() - t0
        nxt = batch[-1] + 1
    span = done.max()
    lat = (done - arrive) * 1e3
    prec = stream_precision_errors(dev, reqs, pool, offs, px, entry)
    n_sat = len(batches(range(n_requests)))
    stream_plans = plan_s[n_sat:]
    return {"workload": f"{n_requests} requests: 256x256 / 512x512 / 1024x768 / 2048x2048 uniform, B 8/16/32, "
                        "C_R ~ U(0.05,0.5), ZZ/BBV/DD; abcs_encode (budget+sense+inverse DCT), plan per batch, "
                        "batches formed by the library's Admission (outputs within the budget, arrival order), "
                        "launch splits from the tuned table",
            "pixels": int(total_px), "batch_budget_bytes": STREAM_BUDGET_BYTES,
            "saturated": {"mpixel_per_s": round(sat_rate / 1e6, 1), "seconds": round(sat_s, 4),
                          "batches": n_sat, "plan_seconds": round(plan_total_s, 4),
                          "mpixel_per_s_with_planning": round(total_px / (sat_s + plan_total_s) / 1e6, 1)},
            "stream": {"offered_load": load, "mpixel_per_s": round(total_px / span / 1e6, 1),
                       "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                                      "p99": round(float(np.percentile(lat, 99)), 3)},
                       "plan_ms_mean": round(1e3 * float(np.mean(stream_plans)), 3) if stream_plans else None},
            "precision_vs_oracle": prec}


def bounds_section(dev, plan, px, k, out, images):
    """Full-sensing bounds on the step's plan (Section IV, Section V-C): time
    of THI and THB per call over all encodings, mean PSNR per C_R of THI, THB
    and the adaptive decodings of the step, and the correlation of THI's
    per-block counts with the BBV / DD budgets (the quantity of Table 2),
    averaged over the images, with the largest p-value of rho = 0."""
    import torch
    import paper_2001_09632_amd as g
    n_img = len(SEEDS)
    ws = torch.empty(g.threshold_workspace_bytes(plan), dtype=torch.uint8, device=dev)
    m = {r: torch.empty(plan.blocks, dtype=torch.int32, device=dev) for r in ("thi", "thb")}
    dec = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    rho = torch.empty(plan.n, dtype=torch.float64, device=dev)
    pval = torch.empty(plan.n, dtype=torch.float64, device=dev)
    ref = torch.from_numpy(images).to(dev).float()

    def psnr(buf):
        x = buf.view(len(METHODS), len(SUBRATES), n_img, H, W).clamp(0, 255)
        mse = ((x - ref[None, None]) ** 2).mean(dim=(3, 4))
        return (10.0 * torch.log10(255.0 ** 2 / mse)).mean(dim=2)  # (method, C_R)

    res = {"encodings": plan.n, "pixels": plan.pixels}
    table = {"bbv": psnr(out)[0].tolist(), "dd": psnr(out)[1].tolist()}
    # L-DCT-ZZ on the same images and subrates (the non-adaptive reference
    # of Section VII-A), and the blocks each rule leaves with no coefficient
    zz_plan = g.Plan([dict(e, method="zz") for e in entries()[:n_img * len(SUBRATES)]], features=())
    kz = torch.empty(zz_plan.blocks, dtype=torch.int32, device=dev)
    oz = torch.empty(zz_plan.blocks, dtype=torch.int64, device=dev)
    sz = torch.empty(zz_plan.blocks, dtype=torch.int32, device=dev)
    yz = torch.empty(zz_plan.meas, dtype=torch.float32, device=dev)
    xz = torch.empty(zz_plan.pixels, dtype=torch.float32, device=dev)
    g.encode(zz_plan, px, kz, oz, sz, yz, xz)
    xz = xz.view(len(SUBRATES), n_img, H, W).clamp(0, 255)
    table["zz"] = (10.0 * torch.log10(255.0 ** 2 / ((xz - ref[None]) ** 2).mean(dim=(2, 3)))).mean(dim=1).tolist()
    nb = (H // B) * (W // B)
    zero = (k.view(len(METHODS), len(SUBRATES), n_img, nb) == 0).sum(dim=3)       # per image
    res["zero_budget_blocks_by_cr"] = {meth: {str(cr): int(zero[i, j].sum()) for j, cr in enumerate(SUBRATES)}
                                       for i, meth in enumerate(METHODS)}
    res["images_with_zero_budget_blocks_by_cr"] = {
        meth: {str(cr): int((zero[i, j] > 0).sum()) for j, cr in enumerate(SUBRATES)} for i, meth in enumerate(METHODS)}
    # the same PSNR table over the images where BBV leaves no block empty at
    # any subrate (the saturated, perfectly flat areas of the other images
    # carry no BBV weight, so those blocks get no coefficient at all)
    clean_img = (zero[0].sum(dim=0) == 0)
    x_ad = out.view(len(METHODS), len(SUBRATES), n_img, H, W)[:, :, clean_img].clamp(0, 255)
    p_ad = (10.0 * torch.log10(255.0 ** 2 / ((x_ad - ref[clean_img][None, None]) ** 2).mean(dim=(3, 4)))).mean(dim=2)
    p_zz = (10.0 * torch.log10(255.0 ** 2 / ((xz[:, clean_img] - ref[clean_img][None]) ** 2).mean(dim=(2, 3)))).mean(dim=1)
    res["psnr_db_by_cr_without_zero_budget_images"] = {
        "images": int(clean_img.sum()),
        "bbv": {str(cr): round(v, 3) for cr, v in zip(SUBRATES, p_ad[0].tolist())},
        "dd": {str(cr): round(v, 3) for cr, v in zip(SUBRATES, p_ad[1].tolist())},
        "zz": {str(cr): round(v, 3) for cr, v in zip(SUBRATES, p_zz.tolist())}}
    for r in ("thi", "thb"):
        g.threshold(plan, px, m[r], dec, rule=r, workspace=ws)
        torch.cuda.synchronize()
        table[r] = psnr(dec)[0].tolist()  # the same for both halves of the plan
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        for _ in range(3):
            g.threshold(plan, px, m[r], dec, rule=r, workspace=ws)
        e[1].record()
        torch.cuda.synchronize()
        ms = e[0].elapsed_time(e[1]) / 3
        res[r + "_ms"] = round(ms, 3)
        res[r + "_mpix_s"] = round(plan.pixels / (ms * 1e-3) / 1e6, 1)
    g.budget_correlation(plan, m["thi"], k, rho, pval)
    r = rho.view(len(METHODS), len(SUBRATES), n_img).nanmean(dim=2).tolist()
    pmax = pval.view(len(METHODS), len(SUBRATES), n_img).amax(dim=2).tolist()
    res["psnr_db_by_cr"] = {name: {str(cr): round(v, 3) for cr, v in zip(SUBRATES, vals)}
                            for name, vals in table.items()}
    res["rho_thi_vs_budget_by_cr"] = {meth: {str(cr): round(v, 4) for cr, v in zip(SUBRATES, r[i])}
                                      for i, meth in enumerate(METHODS)}
    res["p_value_max_by_cr"] = {meth: {str(cr): float("%.3g" % v) for cr, v in zip(SUBRATES, pmax[i])}
                                for i, meth in enumerate(METHODS)}
    return res


def wht_section(dev, px, images, out_dct):
    """Walsh-Hadamard sensing (Section IV's alternative transform) on the same
    640 encodings: time per budget + sense + decode step (vector-ALU kernels)
    and mean PSNR per C_R next to the DCT's."""
    import torch
    import paper_2001_09632_amd as g
    n_img = len(SEEDS)
    plan = g.Plan([dict(e, transform="wht") for e in entries()])
    k = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    off = torch.empty(plan.blocks, dtype=torch.int64, device=dev)
    stat = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    y = torch.empty(plan.meas, dtype=torch.float32, device=dev)
    out = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    ref = torch.from_numpy(images).to(dev).float()

    def step():
        g.budget(plan, px, k, off, stat)
        g.sense(plan, px, k, off, y)
        g.reconstruct(plan, y, k, off, out)

    def psnr(buf):
        x = buf.view(len(METHODS), len(SUBRATES), n_img, H, W).clamp(0, 255)
        mse = ((x - ref[None, None]) ** 2).mean(dim=(3, 4))
        return (10.0 * torch.log10(255.0 ** 2 / mse)).mean(dim=2)

    step()
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    for _ in range(3):
        step()
    e[1].record()
    torch.cuda.synchronize()
    ms = e[0].elapsed_time(e[1]) / 3
    pw, pd = psnr(out).tolist(), psnr(out_dct).tolist()
    return {"ms_per_step": round(ms, 3), "mpix_s": round(plan.pixels / (ms * 1e-3) / 1e6, 1),
            "psnr_db_by_cr": {f"{xf}-{m}": {str(cr): round(v, 3) for cr, v in zip(SUBRATES, tab[i])}
                              for xf, tab in (("wht", pw), ("dct", pd)) for i, m in enumerate(METHODS)}}


def train_section(dev, batch=32, steps=10):
    """Training steps of both learned denoisers on a batch of 32 synthetic
    128x128 crops with Gaussian noise (sigma 25): crops/s and the matrix-core
    roofline of a step (forward + input and weight gradients = 3 x the
    forward convolution flops)."""
    import numpy as np
    import torch
    import paper_2001_09632_amd as g
    from paper_2001_09632_amd.train import he_init, dncnn_init
    import synth
    crop = 128
    plan = g.Plan([dict(height=crop, width=crop, block=16, subrate=0.25, method="zz", pixel_offset=0)
                   for _ in range(batch)])
    clean = np.stack([synth.synth_image(5000 + i, crop, crop).astype(np.float32) for i in range(batch)])
    rng = np.random.default_rng(12)
    x = torch.from_numpy((clean + rng.normal(0, 25, clean.shape)).astype(np.float32).reshape(-1)).to(dev)
    t = torch.from_numpy(clean.reshape(-1)).to(dev)
    sig = torch.full((batch,), 25.0, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    out = {}
    for name, n_mid in (("cnn", 6), ("dncnn", 15)):
        if name == "cnn":
            prm = torch.from_numpy(he_init(0)).to(dev)
            run = None
            ws = torch.empty(g.cnn_train_workspace_bytes(plan), dtype=torch.uint8, device=dev)
        else:
            b0, r0 = dncnn_init(0)
            prm = torch.from_numpy(b0).to(dev)
            run = torch.from_numpy(r0).to(dev)
            ws = torch.empty(g.dncnn_train_workspace_bytes(plan), dtype=torch.uint8, device=dev)
        m, v = torch.zeros_like(prm), torch.zeros_like(prm)

        def step(k):
            if run is None:
                g.cnn_train_step(plan, prm, m, v, k, 1e-4, x, sig, t, loss, workspace=ws)
            else:
                g.dncnn_train_step(plan, prm, m, v, run, k, 1e-4, x, sig, t, loss, workspace=ws)

        for k in range(1, 4):
            step(k)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for k in range(4, 4 + steps):
            step(k)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / steps
        flop = 3 * plan.pixels * 2 * 9 * (2 * 64 + n_mid * 64 * 64 + 64)
        ach = flop / (ms * 1e-3) / 1e12
        out[name] = {"ms_per_step": round(ms, 3), "crops_per_s": round(batch / (ms * 1e-3), 1),
                     "roofline": {"bound": "mfma", "achieved": round(ach, 1), "peak": BF16_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": round(ach / BF16_PEAK_TFLOPS, 4)}}
    out["batch"] = f"{batch} x {crop}x{crop} crops"
    return out


def _oracle_encodings(img):
    """Budget + sensing + decoding of one image at every (estimator, subrate)
    pair by the FP64 oracle, with numpy's BLAS held to one thread; returns
    the pixels encoded."""
    from threadpoolctl import threadpool_limits
    from oracle import abcs as orc
    with threadpool_limits(1):
        for m in METHODS:
            for cr in SUBRATES:
                k, _, y = orc.encode(img, B, cr, orc.METHOD_NAMES[m])
                orc.reconstruct(y, B, k, H, W)
    return len(METHODS) * len(SUBRATES) * img.size


def _pool_ready(_):
    import oracle.abcs  # noqa: F401
    import threadpoolctl  # noqa: F401
    return os.getpid()


def cpu_baseline(images, single_s=10.0):
    """The FP64 oracle (budget + sensing + decoding, numpy) on the host's
    cores: one worker process per core of this process's CPU set, each image's
    ten encodings in one worker, over all 64 images (workers started before
    the clock); and one thread alone on the first images for about
    `single_s` seconds."""
    from concurrent.futures import ProcessPoolExecutor
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    px1, n1 = 0, 0
    while n1 < len(images) and time.perf_counter() - t0 < single_s:
        px1 += _oracle_encodings(images[n1])
        n1 += 1
    dt1 = time.perf_counter() - t0
    with ProcessPoolExecutor(max_workers=cores) as ex:
        list(ex.map(_pool_ready, range(cores)))
        t0 = time.perf_counter()
        pxn = sum(ex.map(_oracle_encodings, list(images)))
        dtn = time.perf_counter() - t0
    return dict(value=pxn / dtn / 1e6, unit="Mpixel/s", cores=cores, kind="oracle",
                sample=f"all 640 image encodings (64 images x 2 estimators x 5 subrates), budget+sense+inverse DCT "
                       f"in float64 numpy, one worker process per core, {dtn:.1f} s",
                single_thread={"value": round(px1 / dt1 / 1e6, 3), "unit": "Mpixel/s",
                               "sample": f"{10 * n1} encodings ({n1} images), {dt1:.1f} s"})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-stream", action="store_true", help="skip the mixed request-stream section")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ida", action="store_true")
    ap.add_argument("--no-bounds", action="store_true", help="skip the THI / THB bounds section")
    ap.add_argument("--no-wht", action="store_true", help="skip the Walsh-Hadamard section")
    ap.add_argument("--no-train", action="store_true", help="skip the denoiser training-step section")
    ap.add_argument("--cnn-weights", default=os.path.join(ROOT, "paper_2001_09632_amd", "weights", "ida_cnn.npy"))
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run a device-to-device copy of this many MiB (5 times) and exit; "
                         "its FETCH_SIZE / WRITE_SIZE readings calibrate the traffic counters")
    ap.add_argument("--denoiser-probe", action="store_true",
                    help="only run abcs_denoise with BM3D and with the CNN on the IDA batch's real-time decodings "
                         "(sigma 25), 3 calls each, and exit: the workload of the denoisers' counter profiles")
    ap.add_argument("--bw-probe", type=float, default=0.0,
                    help="only time a device copy and a fill of this many MiB and print their HBM rates")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the batch would shard by "
              f"image across GPUs with no communication, which this build does not run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2001_09632_amd as g

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe > 0:
        n = int(args.copy_probe * (1 << 20)) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "launches": 5}))
        return
    if args.bw_probe > 0:
        # practical HBM rates of plain torch kernels: a device copy (read +
        # write) and a fill (write only), 10 timed launches each
        n = int(args.bw_probe * (1 << 20)) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        out = {"bytes": 4 * n}
        for name, fn, moved in (("copy", lambda: b.copy_(a), 8 * n), ("fill", lambda: b.fill_(1.5), 4 * n)):
            for _ in range(3):
                fn()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            for _ in range(10):
                fn()
            ev[1].record()
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / 10
            out[name] = {"ms": round(ms, 4), "GB_per_s": round(moved / ms / 1e6, 1)}
        print(json.dumps(out))
        return
    if args.denoiser_probe:
        from paper_2001_09632_amd.train import encode_batch, load_params
        imgs, crs, methods = ida_workload()
        dplan, dy, dk, doff = encode_batch(dev, imgs, crs, methods)
        io = torch.empty(dplan.pixels, dtype=torch.float32, device=dev)
        g.reconstruct(dplan, dy, dk, doff, io)
        sig = torch.full((dplan.n,), 25.0, dtype=torch.float32, device=dev)
        o = torch.empty_like(io)
        prm = torch.from_numpy(load_params(args.cnn_weights)).to(dev)
        rec = {}
        for den, params, reps in (("bm3d", None, 3), ("cnn", prm, 20)):
            ws = torch.empty(g.denoise_workspace_bytes(dplan, den), dtype=torch.uint8, device=dev)
            # untimed calls for half a second first (clocks out of idle)
            t_end = time.perf_counter() + SETTLE_S
            while time.perf_counter() < t_end:
                g.denoise(dplan, io, sig, o, den, params=params, workspace=ws)
                torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            for _ in range(reps):
                g.denoise(dplan, io, sig, o, den, params=params, workspace=ws)
            ev[1].record()
            torch.cuda.synchronize()
            rec[den + "_ms_per_call"] = round(ev[0].elapsed_time(ev[1]) / reps, 3)
        print(json.dumps({"denoiser_probe": rec, "pixels": dplan.pixels}))
        return
    # launch splits of the sensing and decoding kernels: the stored table of
    # this build, or a tuning run now (about a minute) when there is none
    from paper_2001_09632_amd import tune
    t_tune = time.perf_counter()
    table, tune_source = tune.ensure(log=log)
    launch_tuning = {"source": tune_source, "build_id": table["build_id"],
                     "seconds": round(time.perf_counter() - t_tune, 2), "size_classes": table["size_classes"],
                     "splits": tune.splits_summary(table)}

    log("generating images")
    images = make_images()
    px = torch.from_numpy(images.reshape(-1)).to(dev)
    plan = g.Plan(entries())
    k = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    off = torch.empty(plan.blocks, dtype=torch.int64, device=dev)
    stat = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    y = torch.empty(plan.meas, dtype=torch.float32, device=dev)
    out = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        # abcs_encode's two launches, called as its two halves so that each
        # can be timed: phase-1 statistics + apportionment (abcs_budget), then
        # sensing and the decoder in one pass over each tile
        # (abcs_sense_decode)
        if ev is not None:
            ev[0].record(stream)
        g.budget(plan, px, k, off, stat, stream)
        if ev is not None:
            ev[1].record(stream)
        g.sense_decode(plan, px, k, off, y, out, stream)
        if ev is not None:
            ev[2].record(stream)

    # Settle: the GPU leaves its idle clocks only after some hundred
    # milliseconds of work (a step takes 0.24 ms at full clock and about
    # 0.31 ms in the first hundred calls), so the step runs untimed for a fixed
    # SETTLE_S before the warmup steps; reported in the JSON line.
    log("settle")
    settle_steps = 0
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < SETTLE_S:
        for _ in range(50):
            step()
        torch.cuda.synchronize()
        settle_steps += 50
    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    log("timing")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_budget = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    ms_sd = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms_step = elapsed / args.steps * 1e3

    pixels_per_step = plan.pixels
    value = pixels_per_step * args.steps / elapsed / 1e6
    # the dominant launch: sensing + decoding (k_encode16); it moves every
    # byte the step must move (pixels in, y and the decoded images out, k
    # and offsets in), so its algorithmic bytes are the step's as well
    step_bytes = algorithmic_bytes(plan, "sense_decode")
    ach = step_bytes / (ms_sd * 1e-3) / 1e9
    roofline = dict(bound="hbm", kernel="sense_decode (k_encode16)", achieved=round(ach, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4), traffic=measured_traffic("sense_decode"),
                    algorithmic_bytes=step_bytes)
    ach_step = step_bytes / (ms_step * 1e-3) / 1e9
    roofline_step = dict(bound="hbm", achieved=round(ach_step, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=round(ach_step / HBM_PEAK_GBS, 4), algorithmic_bytes=step_bytes,
                         basis="(1 + 4 y/pixel + 4 + 12/B^2) bytes per pixel over ms_per_step")
    per_kernel_ms = dict(budget=round(ms_budget, 4), sense_decode=round(ms_sd, 4))

    # The same step in one launch (abcs_encode with a workspace: statistics,
    # apportionment, sensing and decoding in k_encode_fused, after a fill of
    # its synchronisation words), for comparison; same bits.
    y1, out1 = y.clone(), out.clone()
    ws_enc = torch.empty(max(1, g.encode_workspace_bytes(plan)), dtype=torch.uint8, device=dev)
    assert g.encode_workspace_bytes(plan) > 0, "the step's plan should be eligible for the one-launch encoder"
    e1 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for rep in range(2):
        e1[0].record(stream)
        for _ in range(10):
            g.encode(plan, px, k, off, stat, y, out, stream, workspace=ws_enc)
        e1[1].record(stream)
        torch.cuda.synchronize()
    per_kernel_ms["encode_one_launch"] = round(e1[0].elapsed_time(e1[1]) / 10, 4)
    assert torch.equal(y, y1) and torch.equal(out, out1), "the one-launch encoder differs from the two launches"
    assert int(ws_enc[4:8].view(torch.int32).item()) == 0, "the one-launch encoder's wait gave up"

    # and as three calls (budget, sense, reconstruct: the decoder reads y back)
    y32, out32 = y.clone(), out.clone()
    e3 = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for rep in range(2):
        e3[0].record(stream)
        for _ in range(10):
            g.sense(plan, px, k, off, y, stream)
        e3[1].record(stream)
        for _ in range(10):
            g.reconstruct(plan, y, k, off, out, stream)
        e3[2].record(stream)
        torch.cuda.synchronize()
    per_kernel_ms["sense_alone"] = round(e3[0].elapsed_time(e3[1]) / 10, 4)
    per_kernel_ms["reconstruct_alone"] = round(e3[1].elapsed_time(e3[2]) / 10, 4)
    assert torch.equal(y, y32) and torch.equal(out, out32), "separate calls differ from the fused pass"

    # The 16-bit operand modes of the same transforms (budget unchanged):
    # time per sense_decode call, and the deviation of y and of the decoded
    # images from the float32 path and from the float64 oracle (on a sample
    # of 8 images at every estimator and subrate).  Context only; the
    # headline is float32.
    prec = {}
    y_m = torch.empty_like(y)
    out_m = torch.empty_like(out)
    sample = oracle_decodes(images, plan, k.cpu().numpy())
    prec["fp32"] = precision_errors(plan, out32.cpu().numpy(), sample, images)
    prec["fp32"]["sense_decode_ms"] = round(ms_sd, 4)
    for mode in ("bf16x3", "fp16x3", "bf16", "fp16"):
        g.sense_decode(plan, px, k, off, y_m, out_m, stream, precision=mode)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        for _ in range(5):
            g.sense_decode(plan, px, k, off, y_m, out_m, stream, precision=mode)
        e[1].record(stream)
        torch.cuda.synchronize()
        rec_m = precision_errors(plan, out_m.cpu().numpy(), sample, images)
        rec_m.update({"sense_decode_ms": round(e[0].elapsed_time(e[1]) / 5, 4),
                      "max_abs_dy_vs_fp32": round(float((y_m - y32).abs().max()), 5),
                      "max_abs_dpx_vs_fp32": round(float((out_m - out32).abs().max()), 5)})
        prec[mode] = rec_m

    log("single image")
    single = single_image_section(dev)

    bounds = None
    if not args.no_bounds:
        log("bounds")
        bounds = bounds_section(dev, plan, px, k, out32, images)

    wht = None
    if not args.no_wht:
        log("wht")
        wht = wht_section(dev, px, images, out32)

    train = None
    if not args.no_train:
        log("train")
        train = train_section(dev)

    ida = None
    if not args.no_ida:
        log("ida")
        ida = ida_section(dev, args.cnn_weights)

    stream = None
    if not args.no_stream:
        log("stream")
        stream = stream_section(dev)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(images)

    rec = {
        "metric": "Mpixel/s ABCS sense+iDCT; IDA images/s at matched PSNR, learned vs plain",
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64 synthetic 512x512 uint8 images, B=16, AL-DCT-BBV and AL-DCT-DD at C_R "
                               "0.1/0.2/0.3/0.4/0.5 (640 encodings per step): budget + sense + masked inverse DCT "
                               "(abcs_budget, then abcs_sense_decode: the 2 launches of abcs_encode)",
                   "images": len(SEEDS), "height": H, "width": W, "block": B, "encodings_per_step": plan.n,
                   "pixels_per_step": pixels_per_step},
        "settle": {"seconds": SETTLE_S, "steps": settle_steps},
        "per_kernel_ms": per_kernel_ms,
        "launch_tuning": launch_tuning,
        "precision_modes": prec,
        "single_image": single,
        "roofline": roofline,
        "roofline_step": roofline_step,
        "cpu_baseline": cpu,
        "bounds": bounds,
        "wht": wht,
        "train": train,
        "ida": ida,
        "stream": stream,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
