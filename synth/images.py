"""Seeded synthetic 8-bit greyscale images.

Recipe (all arithmetic in float64, one independent generator per image):

1. background level b ~ U(60, 190);
2. + 20 anisotropic Gaussian blobs: centre uniform over the image,
   sigma_x, sigma_y ~ U(0.02, 0.25) * min(H, W), angle ~ U(0, pi),
   amplitude ~ U(-90, 90);
3. 8 opaque filled star-shaped polygons painted in order: 3..8 vertices at
   sorted random angles, radii r * U(0.5, 1) with r ~ U(0.05, 0.25) * min(H, W),
   grey level ~ U(0, 255), even-odd rule on pixel centres, no anti-aliasing;
4. + 1/f texture: white N(0, 1) noise shaped in the Fourier domain by
   1 / max(|f|, 1 / max(H, W)), DC removed, rescaled to std ~ U(4, 16);
5. clip to [0, 255], round half to even, cast to uint8.

The parameter draws and the texture noise use two separate streams derived
from the image seed, so a change in one does not shift the other.
"""

import numpy as np


def _streams(seed):
    ss = np.random.SeedSequence([int(seed), 0x41424353])
    p, t = ss.spawn(2)
    return np.random.Generator(np.random.PCG64(p)), np.random.Generator(np.random.PCG64(t))


def _polygon_mask(h, w, xs, ys):
    """Even-odd point-in-polygon test on pixel centres (x + 0.5, y + 0.5)."""
    py = (np.arange(h, dtype=np.float64) + 0.5)[:, None]
    px = (np.arange(w, dtype=np.float64) + 0.5)[None, :]
    inside = np.zeros((h, w), dtype=bool)
    n = len(xs)
    for e in range(n):
        x0, y0 = xs[e], ys[e]
        x1, y1 = xs[(e + 1) % n], ys[(e + 1) % n]
        if y0 == y1:
            continue
        crosses = (y0 > py) != (y1 > py)
        xint = x0 + (py - y0) * (x1 - x0) / (y1 - y0)
        inside ^= crosses & (px < xint)
    return inside


def synth_image(seed, height, width):
    """Return one (height, width) uint8 image for `seed`."""
    h, w = int(height), int(width)
    if h <= 0 or w <= 0:
        return np.zeros((max(h, 0), max(w, 0)), dtype=np.uint8)
    rp, rt = _streams(seed)
    s = float(min(h, w))
    yy = np.arange(h, dtype=np.float64)[:, None] + 0.5
    xx = np.arange(w, dtype=np.float64)[None, :] + 0.5

    img = np.full((h, w), rp.uniform(60.0, 190.0), dtype=np.float64)

    for _ in range(20):
        cx, cy = rp.uniform(0.0, w), rp.uniform(0.0, h)
        sx, sy = rp.uniform(0.02, 0.25) * s, rp.uniform(0.02, 0.25) * s
        ang = rp.uniform(0.0, np.pi)
        amp = rp.uniform(-90.0, 90.0)
        ca, sa = np.cos(ang), np.sin(ang)
        dx, dy = xx - cx, yy - cy
        u = ca * dx + sa * dy
        v = -sa * dx + ca * dy
        img += amp * np.exp(-0.5 * ((u / sx) ** 2 + (v / sy) ** 2))

    for _ in range(8):
        nv = int(rp.integers(3, 9))
        cx, cy = rp.uniform(0.0, w), rp.uniform(0.0, h)
        r = rp.uniform(0.05, 0.25) * s
        angs = np.sort(rp.uniform(0.0, 2.0 * np.pi, size=nv))
        rad = r * rp.uniform(0.5, 1.0, size=nv)
        grey = rp.uniform(0.0, 255.0)
        mask = _polygon_mask(h, w, cx + rad * np.cos(angs), cy + rad * np.sin(angs))
        img[mask] = grey

    tex_std = rp.uniform(4.0, 16.0)
    noise = rt.standard_normal((h, w))
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.fftfreq(w)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    spec = np.fft.fft2(noise) / np.maximum(f, 1.0 / max(h, w))
    spec[0, 0] = 0.0
    tex = np.real(np.fft.ifft2(spec))
    sd = tex.std()
    if sd > 0:
        img += tex * (tex_std / sd)

    return np.rint(np.clip(img, 0.0, 255.0)).astype(np.uint8)


def synth_batch(seeds, height, width):
    """Stack of images, one per seed: (len(seeds), height, width) uint8."""
    return np.stack([synth_image(s, height, width) for s in seeds])
