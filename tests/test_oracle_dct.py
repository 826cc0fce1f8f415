"""Pins of the oracle's orthonormal 2D DCT and zigzag order (Section IV)."""
import math
import os

import numpy as np
import pytest
import scipy.fft

from oracle import abcs


@pytest.mark.parametrize("B", [2, 4, 8, 16, 32])
def test_basis_orthonormal(B):
    D = abcs.dct_matrix(B)
    assert np.max(np.abs(D @ D.T - np.eye(B))) < 1e-14


def _brute_dct(X):
    """Direct double-cosine definition of the orthonormal 2D DCT-II."""
    B = X.shape[0]
    out = np.zeros((B, B))
    for u in range(B):
        for v in range(B):
            su = math.sqrt((1.0 if u == 0 else 2.0) / B)
            sv = math.sqrt((1.0 if v == 0 else 2.0) / B)
            acc = 0.0
            for i in range(B):
                for j in range(B):
                    acc += X[i, j] * math.cos((2 * i + 1) * u * math.pi / (2 * B)) * \
                        math.cos((2 * j + 1) * v * math.pi / (2 * B))
            out[u, v] = su * sv * acc
    return out


@pytest.mark.parametrize("B", [2, 4, 8])
def test_block_dct_matches_brute_force(B):
    rng = np.random.default_rng(B)
    X = rng.integers(0, 256, size=(3, B, B)).astype(np.float64)
    C = abcs.block_dct(X, abcs.dct_matrix(B))
    for b in range(3):
        assert np.max(np.abs(C[b] - _brute_dct(X[b]))) < 1e-10


@pytest.mark.parametrize("B", [8, 16, 32])
def test_block_dct_matches_scipy_and_parseval(B):
    rng = np.random.default_rng(100 + B)
    X = rng.integers(0, 256, size=(5, B, B)).astype(np.float64)
    C = abcs.block_dct(X, abcs.dct_matrix(B))
    ref = scipy.fft.dctn(X, type=2, norm="ortho", axes=(1, 2))
    assert np.max(np.abs(C - ref)) < 1e-9
    # Parseval: the orthonormal transform preserves energy (Section V-C)
    assert np.allclose((X ** 2).sum(axis=(1, 2)), (C ** 2).sum(axis=(1, 2)), rtol=1e-13)
    # DC = sum / B
    assert np.allclose(C[:, 0, 0], X.sum(axis=(1, 2)) / B, rtol=1e-14)
    # row index = vertical frequency: a pure horizontal ramp has no energy in u > 0
    ramp = np.tile(np.arange(B, dtype=np.float64), (B, 1))[None]
    Cr = abcs.block_dct(ramp, abcs.dct_matrix(B))[0]
    assert np.max(np.abs(Cr[1:, :])) < 1e-10 and abs(Cr[0, 1]) > 1.0


@pytest.mark.parametrize("B", [4, 8, 16, 32])
def test_block_idct_inverts(B):
    rng = np.random.default_rng(7 + B)
    X = rng.uniform(0, 255, size=(4, B, B))
    D = abcs.dct_matrix(B)
    assert np.max(np.abs(abcs.block_idct(abcs.block_dct(X, D), D) - X)) < 1e-10
    ref = scipy.fft.idctn(X, type=2, norm="ortho", axes=(1, 2))
    assert np.max(np.abs(abcs.block_idct(X, D) - ref)) < 1e-9


def test_zigzag_8x8_is_jpeg(repo_root):
    path = os.path.join(repo_root, "tests", "golden", "jpeg_zigzag_8x8.txt")
    vals = [int(t) for line in open(path) if not line.startswith("#") for t in line.split()]
    assert len(vals) == 64
    assert [r * 8 + c for r, c in abcs.zigzag(8)] == vals


@pytest.mark.parametrize("B", [2, 3, 8, 16, 32])
def test_zigzag_bijection_and_diagonals(B):
    zz = abcs.zigzag(B)
    assert len(zz) == B * B and len(set(zz)) == B * B
    d = [r + c for r, c in zz]
    assert d == sorted(d)
    assert zz[0] == (0, 0)
    if B > 1:
        assert zz[1] == (0, 1) and zz[2] == (1, 0)
