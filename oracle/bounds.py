"""FP64 oracle of the full-sensing bounds THI and THB (Section IV) and of the
correlation study of Section V-C (Table 2).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

Both bounds measure every one of the N = n_B B^2 DCT coefficients and keep M
of them, M = floor(C_R N) as for the sensing algorithms:

  THI(M)  keeps the M coefficients of largest magnitude in the whole image;
          m_i is the number kept in block i.  The DCT preserves inner
          products (Parseval), so no other choice of M coefficients leaves a
          smaller error energy: THI bounds what adaptive 2-D DCT sensing can
          reach (Section V-C).
  THB(M)  keeps, in every block, its k = floor(M / n_B) coefficients of
          largest magnitude.

Readings (the formal definitions are in the paper's supplementary material,
which is not available): ties in magnitude go to the lower block index, then
the lower zigzag rank; the decoded image is the inverse DCT of the kept
coefficients (the others zero).  rho is Pearson's correlation between THI's
m_i and an estimator's per-block budget k_i, and p the probability of the
null hypothesis rho = 0 (two-sided Student t test, the usual test for a
correlation coefficient; the paper reports p below 1e-4 without naming it).

Parity: pinned by tests/test_oracle_bounds.py: exact recovery at C_R = 1,
error energy = sum of dropped c^2, THI <= THB <= L-DCT-ZZ in error energy,
brute-force selection by sorting on a tiny image, and Pearson's rho against
its textbook special cases.
"""

import math

import numpy as np

from . import abcs


def coefficients(img, block):
    """DCT coefficients of every block in zigzag-rank order: (n_B, B^2)."""
    B = int(block)
    D = abcs.dct_matrix(B)
    C = abcs.block_dct(abcs.to_blocks(img, B), D)
    order = abcs.zigzag(B)
    return np.stack([C[:, r, c] for r, c in order], axis=1)


def _decode(coefs, keep, img, block):
    """Inverse DCT of the kept coefficients (rank order) -> (H', W')."""
    B = int(block)
    Hc, Wc, nbx, nby, _ = abcs.geometry(img.shape[0], img.shape[1], B)
    C = np.zeros((coefs.shape[0], B, B))
    for z, (r, c) in enumerate(abcs.zigzag(B)):
        C[:, r, c] = np.where(keep[:, z], coefs[:, z], 0.0)
    return abcs.from_blocks(abcs.block_idct(C, abcs.dct_matrix(B)), nby, nbx)


def total_measurements(img, block, subrate):
    """(M, n_B) with M = floor(C_R N), N = H'W' (as every other rule)."""
    Hc, Wc, _, _, nB = abcs.geometry(img.shape[0], img.shape[1], block)
    N = Hc * Wc
    return int(math.floor(subrate * N)), nB


def thi(img, block, subrate):
    """(m per block, keep mask (n_B, B^2) in rank order, decoded image)."""
    coefs = coefficients(img, block)
    M, nB = total_measurements(img, block, subrate)
    flat = np.abs(coefs).reshape(-1)
    # stable sort on -|c|: equal magnitudes keep index order (block, rank)
    order = np.argsort(-flat, kind="stable")
    keep = np.zeros(flat.size, dtype=bool)
    keep[order[:M]] = True
    keep = keep.reshape(coefs.shape)
    return keep.sum(axis=1).astype(np.int64), keep, _decode(coefs, keep, img, block)


def thb(img, block, subrate):
    """(keep mask, decoded image) with floor(M / n_B) coefficients per block."""
    coefs = coefficients(img, block)
    M, nB = total_measurements(img, block, subrate)
    k = M // nB
    keep = np.zeros(coefs.shape, dtype=bool)
    for i in range(coefs.shape[0]):
        order = np.argsort(-np.abs(coefs[i]), kind="stable")
        keep[i, order[:k]] = True
    return keep, _decode(coefs, keep, img, block)


def pearson_p(rho, n):
    """Two-sided p-value of the null hypothesis rho = 0 for n pairs: the
    Student t statistic t = rho sqrt((n-2)/(1-rho^2)) with n-2 degrees of
    freedom, P(|T| >= |t|) = I_x((n-2)/2, 1/2) with x = 1 - rho^2
    (regularised incomplete beta function)."""
    from scipy.special import betainc
    if not np.isfinite(rho) or n < 3:
        return float("nan")
    nu = n - 2
    x = (1.0 - rho) * (1.0 + rho)
    if x <= 0.0:
        return 0.0
    return float(betainc(nu / 2.0, 0.5, x))


def pearson(a, b):
    """Pearson's correlation coefficient of two equal-length samples."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    da, db = a - a.mean(), b - b.mean()
    den = math.sqrt(float(np.sum(da * da)) * float(np.sum(db * db)))
    return float(np.sum(da * db)) / den if den > 0 else float("nan")
