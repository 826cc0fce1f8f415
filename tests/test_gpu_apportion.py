"""GPU parity of the budget apportionment (eqs 22-23 with the cap rule) on
each of its kernels, chosen by the plan's largest image: up to 2048 and up
to 8192 blocks (blocks in registers), up to 131,072 blocks (on a histogram
of the weights) and beyond (blocks in global memory).  Budgets, statistics
and offsets bit-exact against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import abcs as orc

from gpu_util import Run, pack_images

pytestmark = pytest.mark.gpu


def _check(imgs, reqs, calls=1):
    """calls > 1: the budget runs that many times on one plan (outputs
    refilled between calls), and the last call's outputs are checked."""
    px, d = pack_images(imgs)
    run = Run(px, [dict(d[s], block=B, subrate=cr, method=m) for s, B, cr, m in reqs]).budget()
    for _ in range(calls - 1):
        for t in (run.k, run.off, run.stat):
            t.fill_(-7)
        run.budget()
    run.fetch()
    for j, (s, B, cr, m) in enumerate(reqs):
        got = run.image(j)
        k, stat = orc.budget(imgs[s], B, cr, orc.METHOD_NAMES[m])
        assert np.array_equal(got["stat"], stat), f"stat (request {j}: {imgs[s].shape}, B {B}, C_R {cr}, {m})"
        assert np.array_equal(got["k"], k), f"k (request {j}: {imgs[s].shape}, B {B}, C_R {cr}, {m})"
        assert np.array_equal(got["off"], orc.offsets(k)), f"offsets (request {j})"


@pytest.mark.parametrize("size,B", [((512, 512), 16), ((496, 528), 16), ((400, 656), 16), ((1024, 768), 16), ((1024, 1024), 8), ((2048, 2048), 8)])
def test_apportion_kernels_by_image_size(size, B):
    """Largest images of 1023, 1024, 1025 and 3072 blocks (registers: some
    threads' last blocks empty, or all full), 16,384 and 65,536 blocks
    (histogram), with a small image beside them, so that one plan mixes
    block counts."""
    big = synth.synth_image(4000, *size)
    small = synth.synth_image(4001, 64, 80)
    reqs = [(0, B, 0.1, "bbv"), (0, B, 0.35, "dd"), (0, B, 0.5, "bbv"), (1, 16, 0.2, "dd"), (1, 8, 0.3, "zz")]
    _check([big, small], reqs)


def test_apportion_histogram_kernel_many_weights():
    """73,728 blocks (2048 x 2304 at B = 8), BBV weights spread widely."""
    big = synth.synth_image(4002, 2048, 2304)
    _check([big], [(0, 8, 0.2, "bbv"), (0, 8, 0.45, "dd")], calls=2)


def test_apportion_global_memory_kernel():
    """An image of more than 131,072 blocks (2048 x 4608 at B = 8: 147,456)."""
    big = synth.synth_image(4003, 2048, 4608)
    _check([big], [(0, 8, 0.3, "bbv"), (0, 8, 0.25, "dd")])


def test_apportion_uniform_weights_and_ties():
    """A flat image (every BBV weight 0, so the weights count as equal and
    all remainders tie) and a line pattern (few distinct weights, many equal
    remainders), at several rates."""
    flat = np.full((512, 512), 97, dtype=np.uint8)
    two = np.zeros((256, 512), dtype=np.uint8)
    two[:, ::32] = 255
    two[::48, :] = 200
    reqs = [(0, 16, 0.1, "bbv"), (0, 16, 0.45, "bbv"), (0, 16, 0.3, "dd"), (1, 16, 0.2, "bbv"), (1, 16, 0.25, "dd"),
            (1, 16, 0.4, "dd")]
    _check([flat, two], reqs)


def test_apportion_histogram_ties_across_spans():
    """Images of more than 8192 blocks leave their last pass to many
    workgroups (a span of blocks each): a flat 2048 x 1024 image at B = 8
    (32,768 blocks, every BBV weight 0, so every remainder ties and the
    extra shares run across span and wavefront boundaries), a line pattern
    with few distinct weights, and a large image under ZZ (no
    apportionment) in the same plan.  Three calls on one plan: the weight
    counts these images leave in the plan's tables must not carry over."""
    flat = np.full((2048, 1024), 131, dtype=np.uint8)
    lines = np.zeros((1024, 1536), dtype=np.uint8)
    lines[:, ::40] = 255
    lines[::56, :] = 180
    reqs = [(0, 8, 0.1, "bbv"), (0, 8, 0.37, "bbv"), (0, 8, 0.3, "dd"), (1, 8, 0.2, "bbv"), (1, 8, 0.45, "dd"),
            (1, 16, 0.3, "dd"), (0, 8, 0.25, "zz")]
    _check([flat, lines], reqs, calls=3)


def test_apportion_histogram_weights_beyond_one_wavefront():
    """BBV weights of uniform noise span more than 1024 values, so the passes
    over the weight bins take the workgroup form rather than the
    one-wavefront form: a 2048 x 1024 image at B = 8 (32,768 blocks, passes
    over the blocks on many workgroups) and a 1024 x 512 one (8192 blocks,
    all passes in the histogram kernel) in one plan, at two rates, beside DD
    (few weights: the one-wavefront form)."""
    rng = np.random.default_rng(4004)
    big = rng.integers(0, 256, size=(2048, 1024), dtype=np.uint8)
    mid = rng.integers(0, 256, size=(1024, 512), dtype=np.uint8)
    for img in (big, mid):
        _, stat = orc.budget(img, 8, 0.3, orc.METHOD_NAMES["bbv"])
        assert stat.max() >= 1024, "the weights must span more than one wavefront's bins"
    reqs = [(0, 8, 0.2, "bbv"), (1, 8, 0.2, "bbv"), (0, 8, 0.45, "bbv"), (1, 8, 0.45, "bbv"), (0, 8, 0.3, "dd"),
            (1, 8, 0.3, "dd")]
    _check([big, mid], reqs, calls=2)


def test_apportion_spans_empty_and_ragged():
    """Images just past the 8192-block threshold leave most of their 64
    spans empty: 800 x 656 at B = 8 (8200 blocks, spans of 192, the last 21
    empty) and 1000 x 1032 (16,125 blocks, a ragged last span), BBV and DD,
    two calls on one plan."""
    a = synth.synth_image(4005, 800, 656)
    b = synth.synth_image(4006, 1000, 1032)
    reqs = [(0, 8, 0.25, "bbv"), (0, 8, 0.4, "dd"), (1, 8, 0.15, "bbv"), (1, 8, 0.35, "dd")]
    _check([a, b], reqs, calls=2)
