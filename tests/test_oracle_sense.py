"""Pins of the oracle's sensing operator and masked inverse DCT
(eq 26; real-time decoder of Fig 1)."""
import numpy as np
import pytest

import synth
from oracle import abcs


@pytest.mark.parametrize("method", [abcs.ZZ, abcs.DD])
@pytest.mark.parametrize("B", [8, 16, 32])
def test_exact_recovery_full_subrate(method, B):
    # At C_R = 1 every coefficient of every block is measured and the inverse
    # 2D-DCT returns the block exactly.
    img = synth.synth_image(21, 96, 64)
    k, _, y = abcs.encode(img, B, 1.0, method)
    assert np.all(k == B * B)
    rec = abcs.reconstruct(y, B, k, 96, 64)
    Hc, Wc, *_ = abcs.geometry(96, 64, B)
    assert np.max(np.abs(rec - img[:Hc, :Wc])) < 1e-9


def test_adjoint_is_right_inverse():
    # A A* = I on the measured coefficients (orthonormal rows)
    rng = np.random.default_rng(3)
    k = rng.integers(0, 257, size=12)
    z = rng.normal(size=int(k.sum())) * 50
    x = abcs.sense_adjoint(z, 16, k, 3, 4)
    assert np.max(np.abs(abcs.sense_op(x, 16, k) - z)) < 1e-9
    # <A x, z> = <x, A* z>
    xx = rng.uniform(0, 255, size=(48, 64))
    assert abs(np.dot(abcs.sense_op(xx, 16, k), z) - np.sum(xx * x)) < 1e-6 * np.sum(np.abs(xx * x))


def test_error_energy_is_dropped_coefficients():
    # Parseval on the error: ||I - I_o||^2 equals the energy of the
    # coefficients that were not measured.
    img = synth.synth_image(4, 64, 64)
    k, _, y = abcs.encode(img, 16, 0.2, abcs.BBV)
    rec = abcs.reconstruct(y, 16, k, 64, 64)
    C = abcs.block_dct(abcs.to_blocks(img, 16), abcs.dct_matrix(16))
    total = float(np.sum(C ** 2))
    assert abs(np.sum((rec - img) ** 2) - (total - float(np.sum(y ** 2)))) < 1e-6 * total


def test_nested_masks_do_not_lose_quality():
    img = synth.synth_image(9, 64, 64)
    errs = []
    for kk in (1, 10, 40, 100, 256):
        k = np.full(16, kk)
        y = abcs.sense(img, 16, k)
        errs.append(np.sum((abcs.reconstruct(y, 16, k, 64, 64) - img) ** 2))
    assert all(a >= b - 1e-6 for a, b in zip(errs, errs[1:]))


def test_y_layout_first_coefficients():
    # y starts with block 0's DC, then its (0,1) and (1,0) coefficients
    img = synth.synth_image(2, 32, 32)
    k = np.array([3, 0, 1, 2])
    y = abcs.sense(img, 16, k)
    C = abcs.block_dct(abcs.to_blocks(img, 16), abcs.dct_matrix(16))
    assert y.size == 6
    assert np.allclose(y, [C[0, 0, 0], C[0, 0, 1], C[0, 1, 0], C[2, 0, 0], C[3, 0, 0], C[3, 0, 1]])
    assert np.allclose(abcs.offsets(k), [0, 3, 3, 4])
