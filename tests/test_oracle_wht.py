"""Pins of the Walsh-Hadamard sensing transform of the oracle (Section IV
names the 2-D Walsh-Hadamard transform as the alternative to the DCT)."""
import numpy as np
import pytest
from scipy.linalg import hadamard

import synth
from oracle import abcs


@pytest.mark.parametrize("B", [8, 16, 32])
def test_walsh_is_orthonormal_sequency_ordered(B):
    W = abcs.walsh_matrix(B)
    assert np.allclose(W @ W.T, np.eye(B), atol=1e-14)
    assert np.all(np.abs(np.abs(W) * np.sqrt(B) - 1.0) < 1e-15)
    assert np.all(W[:, 0] > 0)
    # row s changes sign exactly s times
    changes = [int(np.count_nonzero(np.sign(W[s, 1:]) != np.sign(W[s, :-1]))) for s in range(B)]
    assert changes == list(range(B))
    # the rows are those of Sylvester's Hadamard matrix, reordered
    H = hadamard(B) / np.sqrt(B)
    assert sorted(map(tuple, np.round(W * np.sqrt(B)).astype(int))) == sorted(map(tuple, np.round(H * np.sqrt(B)).astype(int)))


def test_walsh_8_textbook_rows():
    # sequency-ordered Walsh functions of length 8 (signs)
    want = ["++++++++", "++++----", "++----++", "++--++--", "+--++--+", "+--+-++-", "+-+--+-+", "+-+-+-+-"]
    W = abcs.walsh_matrix(8)
    got = ["".join("+" if v > 0 else "-" for v in row) for row in W]
    assert got == want


@pytest.mark.parametrize("B", [8, 16, 32])
def test_wht_full_subrate_recovers_and_dc(B):
    img = synth.synth_image(61, 2 * B + 5, 3 * B)
    H, W = img.shape
    k = np.full((H // B) * (W // B), B * B)
    y = abcs.sense(img, B, k, "wht")
    rec = abcs.reconstruct(y, B, k, H, W, "wht")
    assert np.max(np.abs(rec - img[:H // B * B, :W // B * B])) < 1e-9
    # first coefficient of every block = block sum / B
    blocks = abcs.to_blocks(img, B)
    assert np.allclose(y[::B * B], blocks.sum(axis=(1, 2)) / B, rtol=0, atol=1e-9)


def test_wht_coefficients_are_exact_multiples_of_one_over_b():
    """With B = 16 every 2-D coefficient is (1/16) times a sum of +-pixels: exact in float64."""
    img = synth.synth_image(62, 32, 48)
    C = abcs.block_dct(abcs.to_blocks(img, 16), abcs.walsh_matrix(16))
    assert np.array_equal(C * 16, np.round(C * 16))
    # brute force from the +-1 definition for one block
    Wi = np.round(abcs.walsh_matrix(16) * 4).astype(np.int64)
    X = abcs.to_blocks(img, 16)[3].astype(np.int64)
    assert np.array_equal((Wi @ X @ Wi.T), np.round(C[3] * 16).astype(np.int64))


def test_wht_budgets_and_adjoint():
    img = synth.synth_image(63, 64, 80)
    for method in (abcs.ZZ, abcs.BBV, abcs.DD):
        k, _ = abcs.budget(img, 16, 0.25, method, "wht")
        M = int(np.floor(0.25 * 64 * 80))
        if method == abcs.DD:
            assert k.sum() == M
    k, _ = abcs.budget(img, 16, 0.25, abcs.DD, "wht")
    # <A x, z> = <x, A* z>
    rng = np.random.default_rng(2)
    x = rng.standard_normal((64, 80))
    z = rng.standard_normal(int(k.sum()))
    lhs = float(np.dot(abcs.sense_op(x, 16, k, "wht"), z))
    rhs = float(np.sum(x * abcs.sense_adjoint(z, 16, k, 4, 5, "wht")))
    assert lhs == pytest.approx(rhs, rel=1e-12)
