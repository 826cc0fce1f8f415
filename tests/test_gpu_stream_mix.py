"""GPU parity on a seeded sample of the mixed request stream: images of
256x256, 512x512, 1024x768 (W x H) and 2048x2048, subrates drawn from
U(0.05, 0.5), B drawn from {8, 16, 32} and the budget rule from {ZZ, BBV, DD},
all in one plan.  Budgets, statistics and offsets bit-exact; y and decoded
pixels to the same bars as the per-size tests."""
import numpy as np
import pytest

import synth
from oracle import abcs as orc

from gpu_util import Run, pack_images

pytestmark = pytest.mark.gpu

SIZES = [(256, 256), (512, 512), (768, 1024), (2048, 2048)]   # (H, W)
PX_TOL = 1e-3
Y_TOL = {8: 1e-2, 16: 1e-2, 32: 5e-2}


def stream_sample(seed, count):
    """count requests: (image index into a pool of one image per size, B,
    C_R, method); the 2048x2048 size appears once."""
    rng = np.random.default_rng(seed)
    reqs = [(3, 16, 0.3, "dd")]
    while len(reqs) < count:
        s = int(rng.integers(0, 3))
        B = int(rng.choice([8, 16, 32]))
        cr = float(rng.uniform(0.05, 0.5))
        m = str(rng.choice(["zz", "bbv", "dd"]))
        reqs.append((s, B, cr, m))
    return reqs


def test_mixed_stream_sample():
    pool = [synth.synth_image(3000 + i, h, w) for i, (h, w) in enumerate(SIZES)]
    px, d = pack_images(pool)
    reqs = stream_sample(5, 16)
    run = Run(px, [dict(d[s], block=B, subrate=cr, method=m) for s, B, cr, m in reqs]).budget().sense() \
        .reconstruct().fetch()
    for j, (s, B, cr, m) in enumerate(reqs):
        img = pool[s]
        got = run.image(j)
        k, stat = orc.budget(img, B, cr, orc.METHOD_NAMES[m])
        assert np.array_equal(got["k"], k), f"k (request {j}: {img.shape}, B {B}, C_R {cr:.3f}, {m})"
        assert np.array_equal(got["stat"], stat), f"stat (request {j})"
        assert np.array_equal(got["off"], orc.offsets(k)), f"offsets (request {j})"
        y = orc.sense(img, B, k)
        assert np.max(np.abs(got["y"] - y)) < Y_TOL[B], f"y (request {j})"
        rec = orc.reconstruct(got["y"].astype(np.float64), B, k, *img.shape)
        assert np.max(np.abs(got["out"] - rec)) < PX_TOL, f"pixels (request {j})"
