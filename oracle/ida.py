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

Parity: pinned with the identity denoiser against the closed-form scalar
recurrence of each measured coefficient (tests/test_oracle_ida.py).  With a
real denoiser the oracle is the same loop, so it is as pinned as that
denoiser.
"""

import math

import numpy as np

from . import abcs


def identity_denoiser(v, sigma):
    return v


def ida(y, k, block, height, width, iters, damping, denoiser=identity_denoiser,
        trace=None):
    """Run `iters` IDA iterations for one image.

    y       measurements (float, packed as abcs.sense produces them)
    k       per-block coefficient counts
    returns (x^T as a float64 (H', W') array, list of sigma^t)
    `trace`, if a list, receives (t, v^t, sigma^t) for every iteration.
    """
    Hc, Wc, nbx, nby, _ = abcs.geometry(height, width, block)
    y = np.asarray(y, dtype=np.float64)
    m = y.size
    alpha = 1.0 / float(damping)
    x = np.zeros((Hc, Wc), dtype=np.float64)
    z_prev = np.zeros(m, dtype=np.float64)
    sigmas = []
    for t in range(int(iters)):
        r = y - abcs.sense_op(x, block, k)
        z = r + alpha * z_prev
        sigma = math.sqrt(float(np.sum(z * z)) / m) if m else 0.0
        v = x + abcs.sense_adjoint(z, block, k, nby, nbx)
        if trace is not None:
            trace.append((t, v.copy(), sigma))
        x = np.asarray(denoiser(v, sigma), dtype=np.float64)
        z_prev = z
        sigmas.append(sigma)
    return x, sigmas
