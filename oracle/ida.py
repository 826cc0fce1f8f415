"""FP64 oracle of the IDA post-processing loop (Section VI).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

IDA is D-AMP (eqs 13-15) with the Onsager coefficient replaced by the
constant 1/D_F (eq 28).  With r^t = y - A x^t (eq 25), A the block-diagonal
zigzag-DCT operator of eq 26 and m = number of measurements:

    z^t       = r^t + z^{t-1} / D_F
    sigma^t   = ||z^t||_2 / sqrt(m)                     (eq 15)
    v^t       = x^t + A* z^t
    x^{t+1}   = D_{sigma^t}(v^t)                        (eq 13)

started from x^0 = 0 (the ISTA convention stated with eqs 9-10) and z^{-1} = 0,
so z^0 = y, v^0 = A* y = I_o, the real-time reconstruction.  The loop output is
the last denoised iterate x^T; nothing is clipped inside the loop.

D-AMP and DAMP-D (`amp`) keep the Onsager coefficient of eqs 14 / 24 (and
its damped form, eq 27) instead of eq 28's constant:

    alpha^t = div D_{sigma^{t-1}}(v^{t-1}) / m          (D-AMP)
    alpha^t = div D_{sigma^{t-1}}(v^{t-1}) / (m D_F)    (DAMP-D),   alpha^0 = 0

Reading: eq 14 prints both a 1/delta factor and a division by m.  The AMP
correction it generalises (Section III) is (1/delta) times the component mean
of the denoiser's derivative over the N signal components, i.e.
(1/delta)(div / N) = div / m with delta = m / N; that is the coefficient used
here.  The divergence is the Monte-Carlo estimate of D-AMP's authors (ref
[13]): div D(v) ~ b . (D(v + eps b) - D(v)) / eps with eps = max|v| / 1000
(1e-3 when v is 0) and a probe vector b of standard normal values, passed in
and reused at every iteration.

Parity: pinned with the identity denoiser against the closed-form scalar
recurrence of each measured coefficient (tests/test_oracle_ida.py), for IDA
and, with alpha = ||b||^2 / m (the exact Monte-Carlo divergence of the
identity), for D-AMP and DAMP-D; a linear denoiser D(v) = lambda v pins the
divergence path (lambda ||b||^2).  With a real denoiser the oracle is the same
loop, so it is as pinned as that denoiser.
"""

import math

import numpy as np

from . import abcs


def identity_denoiser(v, sigma):
    return v


def bbv_rows(bbv, height, width, block):
    """(a, b, d) of the BBV difference rows: row (e_a - e_b) / sqrt 2 with
    measurement d / sqrt 2, d the signed samples."""
    d, L, X0, nS = bbv
    a, b = abcs.bbv_sample_pairs(height, width, block, L, X0, nS)
    return a, b, np.asarray(d, dtype=np.float64) / math.sqrt(2.0)


def bbv_op(x, a, b):
    """A_bbv x = (x[a] - x[b]) / sqrt 2 (x flattened)."""
    xf = np.asarray(x, dtype=np.float64).reshape(-1)
    return (xf[a] - xf[b]) / math.sqrt(2.0)


def bbv_adjoint(z, a, b, shape):
    """A_bbv* z: +z / sqrt 2 at pixel a, -z / sqrt 2 at pixel b of each row."""
    out = np.zeros(int(np.prod(shape)), dtype=np.float64)
    zs = np.asarray(z, dtype=np.float64) / math.sqrt(2.0)
    np.add.at(out, a, zs)
    np.add.at(out, b, -zs)
    return out.reshape(shape)


def ida(y, k, block, height, width, iters, damping, denoiser=identity_denoiser,
        trace=None, transform="dct", bbv=None):
    """Run `iters` IDA iterations for one image.

    y       measurements (float, packed as abcs.sense produces them)
    k       per-block coefficient counts
    returns (x^T as a float64 (H', W') array, list of sigma^t)
    `trace`, if a list, receives (t, v^t, sigma^t) for every iteration.
    `transform` is the sensing transform of A ("dct" or "wht").
    `bbv`, if given as (samples, L, X0, n_S), adds the BBV samples to A as
    difference rows (e_a - e_b) / sqrt 2 (Section V-A: the phase-1 samples
    may serve as additional reconstruction measurements): their residual
    joins z, A* scatters it back to the two pixels, and m counts them.
    """
    Hc, Wc, nbx, nby, _ = abcs.geometry(height, width, block)
    y = np.asarray(y, dtype=np.float64)
    if bbv is not None:
        ba, bb, bd = bbv_rows(bbv, height, width, block)
    else:
        ba = bb = np.zeros(0, dtype=np.int64)
        bd = np.zeros(0)
    m = y.size + bd.size
    alpha = 1.0 / float(damping)
    x = np.zeros((Hc, Wc), dtype=np.float64)
    z_prev = np.zeros(y.size, dtype=np.float64)
    zb_prev = np.zeros(bd.size, dtype=np.float64)
    sigmas = []
    for t in range(int(iters)):
        r = y - abcs.sense_op(x, block, k, transform)
        z = r + alpha * z_prev
        zb = (bd - bbv_op(x, ba, bb)) + alpha * zb_prev
        sigma = math.sqrt((float(np.sum(z * z)) + float(np.sum(zb * zb))) / m) if m else 0.0
        v = x + abcs.sense_adjoint(z, block, k, nby, nbx, transform)
        if bd.size:
            v = v + bbv_adjoint(zb, ba, bb, v.shape)
        if trace is not None:
            trace.append((t, v.copy(), sigma))
        x = np.asarray(denoiser(v, sigma), dtype=np.float64)
        z_prev = z
        zb_prev = zb
        sigmas.append(sigma)
    return x, sigmas


def amp(y, k, block, height, width, iters, damping, probe, denoiser=identity_denoiser,
        algorithm="damp", transform="dct"):
    """Run `iters` iterations of D-AMP (algorithm "damp", eqs 13-15, 24) or
    DAMP-D ("damp-d", eq 27) for one image.

    probe   the Monte-Carlo probe b, shape (H', W')
    returns (x^T, list of sigma^t, list of alpha^t)
    """
    if algorithm not in ("damp", "damp-d"):
        raise ValueError(algorithm)
    Hc, Wc, nbx, nby, _ = abcs.geometry(height, width, block)
    y = np.asarray(y, dtype=np.float64)
    b = np.asarray(probe, dtype=np.float64).reshape(Hc, Wc)
    m = y.size
    scale = 1.0 if algorithm == "damp" else 1.0 / float(damping)
    x = np.zeros((Hc, Wc), dtype=np.float64)
    z_prev = np.zeros(m, dtype=np.float64)
    alpha = 0.0
    sigmas, alphas = [], []
    for t in range(int(iters)):
        r = y - abcs.sense_op(x, block, k, transform)
        z = r + alpha * z_prev
        sigma = math.sqrt(float(np.sum(z * z)) / m) if m else 0.0
        v = x + abcs.sense_adjoint(z, block, k, nby, nbx, transform)
        x_new = np.asarray(denoiser(v, sigma), dtype=np.float64)
        sigmas.append(sigma)
        alphas.append(alpha)
        if t + 1 < iters:
            vmax = float(np.max(np.abs(v)))
            eps = vmax / 1000.0 if vmax > 0 else 1e-3
            xp = np.asarray(denoiser(v + eps * b, sigma), dtype=np.float64)
            div = float(np.sum(b * (xp - x_new))) / eps
            alpha = scale * div / m if m else 0.0
        x = x_new
        z_prev = z
    return x, sigmas, alphas
