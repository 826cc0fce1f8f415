"""FP64 oracle of the plain BM3D denoiser used inside IDA.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

The paper runs IDA with BM3D (ref [22], Dabov et al., "Image denoising by
sparse 3D transform-domain collaborative filtering") as its non-learned
denoiser (Section VI-4, Fig 7a) but fixes none of its parameters.  This oracle
implements the two-stage method of [22] with the following profile, written
down here because the paper is silent:

  patches           8 x 8 (N1), reference patches every 3 pixels (N_step) in
                    each direction plus the last row / column position, so
                    every pixel is covered
  search window     39 x 39 centred on the reference patch position, clipped
                    to the image (N_S)
  patch distance    d(P, Q) = ||P - Q||^2 / 64 on the stage's input image
  grouping          candidates with d <= tau (stage 1: 2500, stage 2: 400),
                    the reference first, the rest by increasing d, ties to
                    the lower raster index of the patch position; at most
                    N2 (16, 32) members, cut to the largest power of two
  3D transform      orthonormal 8 x 8 DCT-II of every patch, then the
                    orthonormal Haar transform along the group
  stage 1           hard threshold: coefficients with |c| <= 2.7 sigma are set
                    to 0; group weight 1 / (sigma^2 N_har), N_har the number of
                    surviving coefficients (a group with none is weighted as
                    one with N_har = 1)
  stage 2           empirical Wiener shrinkage W = B^2 / (B^2 + sigma^2) with B
                    the 3D spectrum of the same group cut from the stage-1
                    estimate, applied to the group cut from the input; group
                    weight 1 / (sigma^2 max(||W||^2, 2^-16))
  aggregation       every patch estimate is added with its group weight times
                    an 8 x 8 Kaiser window (beta = 2) to a numerator, the weight
                    times the window to a denominator; estimate = num / den
  sigma = 0         returns the input unchanged

Deviations from [22], stated: both stages use the 2D DCT (the 2D bior1.5 of
stage 1 in [22] is replaced); one parameter profile for every sigma (no
switch of N1, tau or lambda above sigma = 40); the two weight floors above
keep every weight finite.

Parity: pinned by tests/test_oracle_bm3d.py: sigma = 0 and constant images
are fixed points, the 3D transform is orthonormal, grouping on a crafted image
reproduces hand-derived groups, the Kaiser window equals its closed form
I0(beta sqrt(1 - t^2)) / I0(beta), both stages' group weights (1 / (sigma^2
N_har) and 1 / (sigma^2 ||W||^2)) reproduce a hand-computed aggregation of
two overlapping single-patch groups (which reduces each stage to 2-D DCT
shrinkage, computed there with scipy's DCT), and the denoiser lowers the
error of a noisy image.  Its absolute quality on natural images is parity unpinned (the paper
gives no BM3D numbers on available data).
"""

import math

import numpy as np

N1 = 8
STEP = 3
HALF_WIN = 19
TAU_HT = 2500.0
TAU_WIE = 400.0
N2_HT = 16
N2_WIE = 32
LAMBDA_3D = 2.7
KAISER_BETA = 2.0
W_FLOOR = 2.0 ** -16


def dct8():
    D = np.empty((N1, N1))
    for u in range(N1):
        s = math.sqrt((1.0 if u == 0 else 2.0) / N1)
        for j in range(N1):
            D[u, j] = s * math.cos(math.pi * (2 * j + 1) * u / (2.0 * N1))
    return D


def kaiser2d():
    k = np.kaiser(N1, KAISER_BETA)
    return np.outer(k, k)


def ref_positions(n):
    """Reference patch origins along one axis of length n (>= 8)."""
    pos = list(range(0, n - N1 + 1, STEP))
    if pos[-1] != n - N1:
        pos.append(n - N1)
    return pos


def haar_fwd(g):
    """Orthonormal Haar transform along axis 0 (length a power of two)."""
    g = np.array(g, dtype=np.float64)
    n = g.shape[0]
    out = g.copy()
    m = n
    while m > 1:
        a = (out[0:m:2] + out[1:m:2]) / math.sqrt(2.0)
        d = (out[0:m:2] - out[1:m:2]) / math.sqrt(2.0)
        out[: m // 2] = a
        out[m // 2: m] = d
        m //= 2
    return out


def haar_inv(h):
    h = np.array(h, dtype=np.float64)
    n = h.shape[0]
    out = h.copy()
    m = 2
    while m <= n:
        a = out[: m // 2].copy()
        d = out[m // 2: m].copy()
        out[0:m:2] = (a + d) / math.sqrt(2.0)
        out[1:m:2] = (a - d) / math.sqrt(2.0)
        m *= 2
    return out


def transform3d(group, D):
    """group (n, 8, 8) -> 3D spectrum: 2D DCT of each patch, Haar along n."""
    spec2 = np.einsum("ur,nrc,vc->nuv", D, group, D)
    return haar_fwd(spec2)


def inverse3d(spec, D):
    spec2 = haar_inv(spec)
    return np.einsum("ur,nuv,vc->nrc", D, spec2, D)


def match(img, ry, rx, tau, n2):
    """Group of the reference patch at (ry, rx): list of patch origins."""
    H, W = img.shape
    y0, y1 = max(0, ry - HALF_WIN), min(H - N1, ry + HALF_WIN)
    x0, x1 = max(0, rx - HALF_WIN), min(W - N1, rx + HALF_WIN)
    ref = img[ry:ry + N1, rx:rx + N1]
    win = np.lib.stride_tricks.sliding_window_view(img[y0:y1 + N1, x0:x1 + N1], (N1, N1))
    d = np.sum((win - ref) ** 2, axis=(2, 3)) / float(N1 * N1)   # (ny, nx)
    qy, qx = np.nonzero(d <= tau)
    qy, qx = qy + y0, qx + x0
    dd = d[qy - y0, qx - x0]
    is_ref = (qy == ry) & (qx == rx)
    order = np.lexsort((qy * W + qx, dd, ~is_ref))      # reference, then d, then raster index
    sel = order[:n2]
    n = 1 << (len(sel).bit_length() - 1)
    sel = sel[:n]
    return [(int(qy[i]), int(qx[i])) for i in sel]


def _aggregate(num, den, positions, est, weight, K):
    for (py, px), e in zip(positions, est):
        num[py:py + N1, px:px + N1] += weight * K * e
        den[py:py + N1, px:px + N1] += weight * K


def stage1(v, sigma, trace=None):
    v = np.asarray(v, dtype=np.float64)
    H, W = v.shape
    D, K = dct8(), kaiser2d()
    num, den = np.zeros_like(v), np.zeros_like(v)
    thr = LAMBDA_3D * sigma
    for ry in ref_positions(H):
        for rx in ref_positions(W):
            pos = match(v, ry, rx, TAU_HT, N2_HT)
            if trace is not None:
                trace[(ry, rx)] = pos
            g = np.stack([v[py:py + N1, px:px + N1] for py, px in pos])
            spec = transform3d(g, D)
            spec[np.abs(spec) <= thr] = 0.0
            nhar = int(np.count_nonzero(spec))
            w = 1.0 / (sigma * sigma * max(nhar, 1))
            _aggregate(num, den, pos, inverse3d(spec, D), w, K)
    return num / den


def stage2(v, basic, sigma):
    v = np.asarray(v, dtype=np.float64)
    basic = np.asarray(basic, dtype=np.float64)
    H, W = v.shape
    D, K = dct8(), kaiser2d()
    num, den = np.zeros_like(v), np.zeros_like(v)
    s2 = sigma * sigma
    for ry in ref_positions(H):
        for rx in ref_positions(W):
            pos = match(basic, ry, rx, TAU_WIE, N2_WIE)
            gb = np.stack([basic[py:py + N1, px:px + N1] for py, px in pos])
            gn = np.stack([v[py:py + N1, px:px + N1] for py, px in pos])
            tb = transform3d(gb, D)
            wie = tb * tb / (tb * tb + s2)
            w = 1.0 / (s2 * max(float(np.sum(wie * wie)), W_FLOOR))
            _aggregate(num, den, pos, inverse3d(wie * transform3d(gn, D), D), w, K)
    return num / den


def bm3d(v, sigma):
    """Two-stage BM3D estimate of the image v (float64 H x W, both >= 8)."""
    v = np.asarray(v, dtype=np.float64)
    if sigma <= 0.0:
        return v.copy()
    basic = stage1(v, sigma)
    return stage2(v, basic, sigma)
