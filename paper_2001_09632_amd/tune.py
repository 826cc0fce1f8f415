"""Launch tuning of the sensing and decoding kernels on the GPU this process
runs on.

The kernels give each tile (up to 16 adjacent blocks of one block row) to one
wavefront; a launch split s gives it to 2^s wavefronts instead
(abcs_set_launch_table).  For every launch kind (block size, transform,
precision) and size class this module times abcs_sense_decode on a batch of
that size at each split (abcs_time_splits), keeps the fastest (split 0 unless
another one is faster by more than TIE), and stores the table in
tuned_launch.json next to the library, under the library's build id (a hash of
its sources' code, comments left out, and compiler flags).  The binding installs that table when it
loads the library; a table stored under another build id is never used: any
change to the kernels or flags asks for a new tuning run.

Timing inputs: seeded smooth random images (the splits' times depend on the
images only through the budgets' spread over the blocks), budgets from the
library's own estimators, rules and subrates cycling over ZZ / BBV / DD and
C_R 0.1 ... 0.5.

    python -m paper_2001_09632_amd.tune [--out PATH] [--reps N]
"""
import argparse
import json
import os
import time

import numpy as np

from . import api

PKG = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(PKG, "tuned_launch.json")
TIE = 0.03
SPLITS = (0, 1, 2)
SIZE_CLASSES = ("< 256 tiles", "< 2048 tiles", "< 16384 tiles", ">= 16384 tiles")
# (images, side) per block size and size class: a side x side image holds
# (side / B) block rows of ceil(side / (16 B)) tiles.
BATCHES = {
    8: ((1, 256), (4, 512), (32, 512), (96, 512)),
    16: ((2, 512), (16, 512), (128, 512), (384, 512)),
    32: ((8, 512), (64, 512), (512, 512), (1536, 512)),
}
POOL = 16            # distinct images behind the descriptors of a batch
KINDS = [(b, "dct", p) for b in (8, 16, 32) for p in api.PRECISIONS] + [(b, "wht", "fp32") for b in (8, 16, 32)]


def smooth_images(n, side, seed=11):
    """n seeded side x side uint8 images: low-pass filtered noise plus a
    gradient (edges and flat areas in varying amounts)."""
    rng = np.random.default_rng(seed)
    f = np.fft.fftfreq(side)
    r2 = f[:, None] ** 2 + f[None, :] ** 2
    out = np.empty((n, side, side), np.uint8)
    for i in range(n):
        cut = rng.uniform(0.01, 0.08)
        spec = np.fft.fft2(rng.normal(size=(side, side))) * np.exp(-r2 / (2 * cut * cut))
        x = np.real(np.fft.ifft2(spec))
        x = (x - x.mean()) / (x.std() + 1e-9)
        yy, xx = np.mgrid[0:side, 0:side] / side
        img = 128 + 45 * x + rng.uniform(-40, 40) * (yy - 0.5) + rng.uniform(-40, 40) * (xx - 0.5)
        out[i] = np.clip(np.rint(img), 0, 255).astype(np.uint8)
    return out


def _batch(dev, block, transform, n, side, px):
    import torch
    rules = ("zz", "bbv", "dd")
    ents = []
    for i in range(n):
        cr = 0.1 + 0.1 * (i % 5)
        rule = rules[(i // 5) % 3]
        if rule == "bbv":
            cr = min(cr, 0.5)
        ents.append(dict(height=side, width=side, row_pitch=side, block=block, subrate=cr, method=rule,
                         transform=transform, pixel_offset=(i % POOL) * side * side))
    plan = api.Plan(ents, features=())
    k = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    off = torch.empty(plan.blocks, dtype=torch.int64, device=dev)
    st = torch.empty(plan.blocks, dtype=torch.int32, device=dev)
    y = torch.empty(max(1, plan.meas), dtype=torch.float32, device=dev)
    out = torch.empty(plan.pixels, dtype=torch.float32, device=dev)
    api.budget(plan, px, k, off, st)
    return plan, k, off, y, out


def tune(reps=10, log=print):
    """Time every launch kind and size class; returns the table (a dict)."""
    import torch
    dev = torch.device("cuda:0")
    api.set_launch_table([])
    entries = []
    t0 = time.perf_counter()
    pools = {}
    for block in (8, 16, 32):
        for sc, (n, side) in enumerate(BATCHES[block]):
            if side not in pools:
                pools[side] = torch.from_numpy(smooth_images(POOL, side).reshape(-1)).to(dev)
            px = pools[side]
            for transform in ("dct", "wht"):
                plan, k, off, y, out = _batch(dev, block, transform, n, side, px)
                got = api.plan_size_class(plan, block, transform)
                assert got == sc, (block, transform, n, side, got, sc)
                for (b, tr, prec) in KINDS:
                    if b != block or tr != transform:
                        continue
                    ms = api.time_splits(plan, px, k, off, y, out, prec, reps)
                    best = 0
                    for s in SPLITS[1:]:
                        if ms[s] < ms[best] * (1 - TIE):
                            best = s
                    entries.append(dict(block=block, transform=transform, precision=prec, size_class=sc,
                                        split=best, ms=[round(v, 5) for v in ms], images=n, side=side))
                    log(f"B {block} {transform} {prec:7s} class {sc}: ms {['%.4f' % v for v in ms]} -> split {best}")
                del plan, k, off, y, out
                torch.cuda.empty_cache()
    props = torch.cuda.get_device_properties(dev)
    return {"build_id": api.build_id(), "device": props.name, "reps": reps, "tie": TIE,
            "size_classes": list(SIZE_CLASSES), "seconds": round(time.perf_counter() - t0, 1), "entries": entries}


def install(table):
    api.set_launch_table([e for e in table["entries"] if e["split"] != 0])


def load(path=CACHE, install_table=True):
    """The stored table for this build (installed into the library), or None
    when there is none or it belongs to another build."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    if table.get("build_id") != api.build_id():
        return None
    if install_table:
        install(table)
    return table


def ensure(path=CACHE, reps=10, log=print):
    """load(), or tune, store and install: (table, 'cache' | 'tuned')."""
    table = load(path)
    if table is not None:
        return table, "cache"
    table = tune(reps=reps, log=log)
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    install(table)
    return table, "tuned"


def splits_summary(table):
    """{'B16/dct/fp32': [split per size class], ...}"""
    out = {}
    for e in table["entries"]:
        key = f"B{e['block']}/{e['transform']}/{e['precision']}"
        out.setdefault(key, [None] * len(SIZE_CLASSES))[e["size_class"]] = e["split"]
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    table = tune(reps=args.reps)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(splits_summary(table)))


if __name__ == "__main__":
    main()
