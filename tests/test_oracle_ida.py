"""Pins of the IDA oracle (Section VI, eqs 13, 15, 25, 28).

With the identity denoiser x^{t+1} = x^t + A* z^t, so every measured
coefficient c of x follows the scalar recurrence (y its measurement,
alpha = 1/D_F):
    z^t = y - c^t + alpha z^{t-1},   c^{t+1} = c^t + z^t,   c^0 = 0, z^{-1} = 0.
Worked by hand, c^t / y for t = 1..8 is
    alpha = 1/2 : 1, 1.5, 1.25, 0.875, 0.8125, 0.96875, 1.078125, ...
    alpha = 1   : 1, 2, 2, 1, 0, 0, 1, 2       (period 6: D_F = 1 oscillates)
    alpha = 0   : 1, 1, 1, ...                   (ISTA fixed point I_o)
and z^t / y for alpha = 1/2 is 1, 0.5, -0.25, -0.375, -0.0625, 0.15625.
"""
import math

import numpy as np
import pytest

import synth
from oracle import abcs, ida

HALF = [1.0, 1.5, 1.25, 0.875, 0.8125, 0.96875, 1.078125]
ONE = [1.0, 2.0, 2.0, 1.0, 0.0, 0.0, 1.0, 2.0]
Z_HALF = [1.0, 0.5, -0.25, -0.375, -0.0625, 0.15625]


@pytest.fixture(scope="module")
def case():
    img = synth.synth_image(31, 64, 48)
    k, _, y = abcs.encode(img, 16, 0.25, abcs.BBV)
    return img, k, y


@pytest.mark.parametrize("damping,ratios", [(2.0, HALF), (1.0, ONE), (math.inf, [1.0] * 5)])
def test_identity_denoiser_recurrence(case, damping, ratios):
    img, k, y = case
    for t, ratio in enumerate(ratios, start=1):
        x, _ = ida.ida(y, k, 16, 64, 48, t, damping)
        c = abcs.sense_op(x, 16, k)
        assert np.max(np.abs(c - ratio * y)) < 1e-8 * np.max(np.abs(y))


def test_sigma_trace_and_first_iterate(case):
    img, k, y = case
    trace = []
    _, sig = ida.ida(y, k, 16, 64, 48, 6, 2.0, trace=trace)
    base = math.sqrt(float(np.sum(y * y)) / y.size)
    assert np.allclose(sig, [abs(r) * base for r in Z_HALF], rtol=1e-9)
    # v^0 = A* y = I_o, the real-time reconstruction
    assert np.max(np.abs(trace[0][1] - abcs.reconstruct(y, 16, k, 64, 48))) < 1e-9


def test_iterates_stay_in_measured_subspace(case):
    img, k, y = case
    x, _ = ida.ida(y, k, 16, 64, 48, 5, 2.0)
    C = abcs.block_dct(abcs.to_blocks(x, 16), abcs.dct_matrix(16))
    zz = abcs.zigzag(16)
    for i, ki in enumerate(k):
        for z in range(int(ki), 256):
            r, c = zz[z]
            assert abs(C[i, r, c]) < 1e-8


def _recurrence_ratios(alpha, steps):
    """c^t / y for t = 1..steps with z^0 = y, c^1 = y and, from t = 1 on,
    z^t = (y - c^t) + alpha z^{t-1}, c^{t+1} = c^t + z^t (y = 1)."""
    c, z_prev, out = 0.0, 0.0, []
    for t in range(steps):
        a = 0.0 if t == 0 else alpha
        z = (1.0 - c) + a * z_prev
        c += z
        z_prev = z
        out.append(c)
    return out


@pytest.mark.parametrize("algorithm,damping", [("damp", 2.0), ("damp-d", 2.0), ("damp-d", 8.0)])
def test_amp_identity_follows_recurrence(case, algorithm, damping):
    """Identity denoiser: the Monte-Carlo divergence is exactly ||b||^2, so
    alpha^t = ||b||^2 / m (/ D_F) from t = 1 on and every measured
    coefficient follows the scalar recurrence."""
    img, k, y = case
    rng = np.random.default_rng(3)
    b = rng.standard_normal(img.shape)
    steps = 4
    m = y.size
    a = float(np.sum(b * b)) / m / (1.0 if algorithm == "damp" else damping)
    for t in range(1, steps + 1):
        x, _, alphas = ida.amp(y, k, 16, 64, 48, t, damping, b, algorithm=algorithm)
        assert alphas[0] == 0.0
        assert np.allclose(alphas[1:], a, rtol=1e-9)
        c = abcs.sense_op(x, 16, k)
        ratio = _recurrence_ratios(a, t)[-1]
        assert np.allclose(c, ratio * y, rtol=1e-9, atol=1e-6 * max(1.0, abs(ratio)) * np.max(np.abs(y)))


def test_amp_linear_denoiser_divergence(case):
    """D(v) = lambda v: div = lambda ||b||^2, so alpha^1 = lambda ||b||^2 / m."""
    img, k, y = case
    b = np.random.default_rng(4).standard_normal(img.shape)
    lam = 0.75
    _, _, alphas = ida.amp(y, k, 16, 64, 48, 2, 2.0, b, denoiser=lambda v, s: lam * v)
    assert math.isclose(alphas[1], lam * float(np.sum(b * b)) / y.size, rel_tol=1e-9)


def test_damp_d_infinite_damping_is_ida_without_memory(case):
    """DAMP-D with D_F = inf has alpha = 0: the same iterates as IDA at D_F = inf."""
    img, k, y = case
    b = np.random.default_rng(5).standard_normal(img.shape)
    xa, sa, _ = ida.amp(y, k, 16, 64, 48, 5, math.inf, b, denoiser=lambda v, s: 0.9 * v, algorithm="damp-d")
    xi, si = ida.ida(y, k, 16, 64, 48, 5, math.inf, denoiser=lambda v, s: 0.9 * v)
    assert np.allclose(xa, xi, rtol=0, atol=1e-9) and np.allclose(sa, si, rtol=1e-12)


# ---------------------------------------------------------------------------
# BBV samples as extra difference rows of A (Section V-A)
# ---------------------------------------------------------------------------

def _bbv_case(seed=21, H=64, W=80, cr=0.2):
    img = synth.synth_image(seed, H, W)
    s = abcs.budget_scalars(H, W, 16, cr, abcs.BBV)
    return img, s


def test_bbv_samples_rebuild_the_statistic():
    img, s = _bbv_case()
    L, X0, nS = s["L"], s["X0"], s["nS"]
    d = abcs.bbv_samples(img, 16, L, X0, nS)
    nbx, nby, nB = 5, 4, 20
    assert d.size == 2 * nS * nB + nS * (nbx + nby)
    a, b = abcs.bbv_sample_pairs(64, 80, 16, L, X0, nS)
    assert np.all((a - b == 1) | (a - b == 80))
    # BBV_i = own top + own left + top of the block below (own bottom edge in
    # the last row) + left of the block to the right (own right edge)
    ad = np.abs(d)
    top = ad[:2 * nS * nB].reshape(nB, 2, nS)[:, 0].sum(axis=1).reshape(nby, nbx)
    left = ad[:2 * nS * nB].reshape(nB, 2, nS)[:, 1].sum(axis=1).reshape(nby, nbx)
    bottom_edge = ad[2 * nS * nB:2 * nS * nB + nS * nbx].reshape(nbx, nS).sum(axis=1)
    right_edge = ad[2 * nS * nB + nS * nbx:].reshape(nby, nS).sum(axis=1)
    below = np.vstack([top[1:], bottom_edge[None, :]])
    right = np.hstack([left[:, 1:], right_edge[:, None]])
    want = (top + left + below + right).reshape(-1)
    assert np.array_equal(want, abcs.bbv_stat(img, 16, L, X0, nS))


def test_bbv_rows_operator_and_adjoint():
    img, s = _bbv_case()
    d = abcs.bbv_samples(img, 16, s["L"], s["X0"], s["nS"])
    a, b, dm = ida.bbv_rows((d, s["L"], s["X0"], s["nS"]), 64, 80, 16)
    # the rows measure the image exactly
    assert np.allclose(ida.bbv_op(img.astype(np.float64), a, b), dm, rtol=0, atol=1e-12)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((64, 80))
    z = rng.standard_normal(d.size)
    assert float(np.dot(ida.bbv_op(x, a, b), z)) == pytest.approx(float(np.sum(x * ida.bbv_adjoint(z, a, b, x.shape))), rel=1e-12)


def test_ida_with_bbv_rows_first_iterate_and_sigma():
    """x0 = 0: z0 = [y; d / sqrt 2], sigma0 = sqrt((|y|^2 + |d|^2 / 2) / (m + M_BBV)),
    and with the identity denoiser x1 = I_o plus d / 2 added at the later and
    subtracted at the earlier pixel of every sample."""
    img, s = _bbv_case()
    k, _ = abcs.budget(img, 16, 0.2, abcs.BBV)
    y = abcs.sense(img, 16, k)
    d = abcs.bbv_samples(img, 16, s["L"], s["X0"], s["nS"])
    x1, sig = ida.ida(y, k, 16, 64, 80, 1, 2.0, bbv=(d, s["L"], s["X0"], s["nS"]))
    want_sigma = math.sqrt((float(np.sum(y * y)) + float(np.sum(d.astype(np.float64) ** 2)) / 2) / (y.size + d.size))
    assert sig[0] == pytest.approx(want_sigma, rel=1e-12)
    want = abcs.reconstruct(y, 16, k, 64, 80).reshape(-1)
    a, b = abcs.bbv_sample_pairs(64, 80, 16, s["L"], s["X0"], s["nS"])
    for ai, bi, di in zip(a, b, d):
        want[ai] += di / 2.0
        want[bi] -= di / 2.0
    assert np.max(np.abs(x1.reshape(-1) - want)) < 1e-9
    # without samples the loop is unchanged
    x_plain, _ = ida.ida(y, k, 16, 64, 80, 3, 2.0)
    x_none, _ = ida.ida(y, k, 16, 64, 80, 3, 2.0, bbv=None)
    assert np.array_equal(x_plain, x_none)
