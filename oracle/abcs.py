"""FP64 oracle for block DCT sensing with BBV / DD adaptive budgets.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path imports this module.

Everything here is written from the paper's definitions, in float64 and
exact integers, with explicit loops over the summation index so that the order
of every floating-point sum is fixed:

  geometry         crop and partition into B x B blocks (eq 20; Alg 1/2 step 1)
  budget_scalars   N, M, C_F, L, X0, n_S, M_BBV, m1, T, pool, cap
                   (eqs 16-18, 21; Alg 2 step 2; Table 1)
  dct_matrix       orthonormal DCT-II basis D (B x B)
  walsh_matrix     orthonormal Walsh-Hadamard basis in sequency order (the
                   alternative sensing transform named in Section IV)
  zigzag           JPEG zigzag scan order of a B x B block (Section IV)
  block_dct        C = D X D^T per block, fixed summation order
  block_idct       X = D^T C D per block
  bbv_stat         block boundary variation, eq 19 with edge rule
  bbv_samples      the signed samples behind eq 19 (extra measurements)
  dd_stat          n_i = #{first m1 zigzag coefficients with |c| > T}
  apportion        capped largest-remainder split (eqs 22-23 with the cap
                   and redistribution rule stated after eq 22)
  budget           per-block coefficient counts k_i for ZZ / BBV / DD
  sense            y: first k_i zigzag coefficients of each block
  reconstruct      masked inverse 2D-DCT (real-time decoder, Fig 1)
  sense_op / sense_adjoint   A x and A* z of the block-diagonal operator (eq 26)

Readings where the paper is silent or garbled (each is also listed in the
design notes):
  * M = floor(C_R * N) with N the cropped pixel count; C_F = N / M.
  * n_S follows eq 18 (floor(B / L)), not the floor(B / C_F) of Alg 1 step 2,
    because the sample positions of eq 19 advance by L.
  * eq 19 indices are 1-based inside the block, row/column B+1 being the first
    row/column of the neighbour below/right.  The differences run along the
    border row (column).  Blocks in the last block row (column) use their own
    last row (column) instead of the missing neighbour.
  * M_BBV counts the samples actually taken: 2 n_S n_B + n_S (n_bx + n_by)
    (eq 21 writes (H + W) / L, which is not an integer unless L divides B).
  * BBV with L < 2 (C_R > 0.5) is outside the method's domain: X0 = 0 would
    place the first difference outside the block.
  * n_S = 0 makes BBV non-adaptive: the budgets are exactly L-DCT-ZZ's.
  * L-DCT-ZZ takes k = floor(B^2 C_R) per block (the per-block m of eq 26);
    the few coefficients this leaves of M are not topped up.
  * DD pool is M - n_B m1 so that every coefficient of the budget is used;
    eq 23's n_B m1 is the same number up to the floor in m1.
  * DD counts the DC coefficient, compares strictly (|c| > T) on raw [0, 255]
    pixels, and picks T from Table 1 by the cropped height: the H = 256 column
    below 512 rows, the H = 512 column otherwise.
  * Apportionment: floor shares; any block whose share reaches its cap is
    fixed at the cap and the rest of the pool is re-split over the other
    blocks; once no cap is hit, the leftover R = P - sum(floors) goes, one
    each, to the R blocks with the largest remainder (P w_i) mod S, ties to
    the lower block index.  If all weights are zero the split is uniform.
  * Blocks are numbered in raster order; y holds each block's coefficients in
    zigzag order, blocks one after the other.

Parity: pinned by tests/test_oracle_*.py against the DCT's closed forms
(orthonormality, Parseval, DC = sum / B), the brute-force cosine definition,
scipy's orthonormal DCT-II, the JPEG zigzag table, exact rational brute force
of the apportionment, hand-computed BBV values and exact recovery at C_R = 1.
"""

import math

import numpy as np

ZZ, BBV, DD = 0, 1, 2
METHOD_NAMES = {"zz": ZZ, "bbv": BBV, "dd": DD}


class DomainError(ValueError):
    """Parameters outside the method's domain (e.g. BBV with C_R > 0.5)."""


# ---------------------------------------------------------------------------
# Geometry and scalars
# ---------------------------------------------------------------------------

def geometry(height, width, block):
    """Crop to whole blocks and count them (eq 20; Alg 1/2 step 1).

    Returns (H', W', n_bx, n_by, n_B) with H' = B floor(H/B), W' = B floor(W/B).
    """
    B = int(block)
    n_by, n_bx = int(height) // B, int(width) // B
    return n_by * B, n_bx * B, n_bx, n_by, n_bx * n_by


def dd_threshold(cropped_height, cf):
    """T from Table 1 (pixel range [0, 255]).

    Columns: H = 256 for cropped heights below 512, H = 512 otherwise.
    """
    if cf <= 2.0:
        return 15
    upper = 3.33 if cropped_height < 512 else 10.0
    return 30 if cf < upper else 60


def budget_scalars(height, width, block, subrate, method):
    """All per-image scalars of the budget, as a dict.

    N   cropped pixel count (eq 20)
    M   floor(C_R N) total measurements
    CF  N / M (compression factor)
    kz  floor(B^2 C_R), the L-DCT-ZZ per-block count (eq 26)
    BBV: L = floor(C_F) (eq 16), X0 = floor(L/2) (eq 17), nS = floor(B/L)
         (eq 18), M_BBV (eq 21, counted), pool = M - M_BBV, cap = B^2 - 2 nS
    DD:  m1 = floor(B^2 / (2 C_F)) (Alg 2 step 2), T (Table 1),
         pool = M - n_B m1, cap = B^2 - m1
    `mode` is the budget actually applied: BBV with nS = 0 reverts to ZZ.
    """
    B = int(block)
    Hc, Wc, nbx, nby, nB = geometry(height, width, B)
    N = Hc * Wc
    cr = float(subrate)
    if not (cr > 0.0 and cr <= 1.0):
        raise DomainError("subrate must be in (0, 1]")
    M = int(math.floor(cr * N))
    if nB == 0 or M == 0:
        raise DomainError("no blocks or no measurements")
    cf = N / M
    s = dict(B=B, Hc=Hc, Wc=Wc, nbx=nbx, nby=nby, nB=nB, N=N, M=M, CF=cf,
             kz=int(math.floor(B * B * cr)), method=int(method), mode=ZZ)
    if method == ZZ:
        return s
    if method == BBV:
        L = int(math.floor(cf))
        if L < 2:
            raise DomainError("BBV needs L = floor(C_F) >= 2 (C_R <= 0.5)")
        X0 = L // 2
        nS = B // L
        s.update(L=L, X0=X0, nS=nS)
        if nS == 0:
            return s
        m_bbv = 2 * nS * nB + nS * (nbx + nby)
        pool = M - m_bbv
        if pool < 0:
            raise DomainError("BBV samples exceed the measurement budget")
        s.update(mode=BBV, M_BBV=m_bbv, pool=pool, cap=B * B - 2 * nS)
        return s
    if method == DD:
        m1 = int(math.floor(B * B / (2.0 * cf)))
        T = dd_threshold(Hc, cf)
        pool = M - nB * m1
        s.update(mode=DD, m1=m1, T=T, pool=pool, cap=B * B - m1)
        return s
    raise ValueError("unknown method")


# ---------------------------------------------------------------------------
# Transform and scan order
# ---------------------------------------------------------------------------

def dct_matrix(block):
    """Orthonormal DCT-II basis: D[u, j] = s_u cos((2j + 1) u pi / (2B)),
    s_0 = sqrt(1/B), s_u = sqrt(2/B).  Built element by element with libm cos.
    """
    B = int(block)
    D = np.empty((B, B), dtype=np.float64)
    for u in range(B):
        s = math.sqrt(1.0 / B) if u == 0 else math.sqrt(2.0 / B)
        for j in range(B):
            D[u, j] = s * math.cos(math.pi * (2 * j + 1) * u / (2.0 * B))
    return D


def walsh_matrix(block):
    """Orthonormal Walsh-Hadamard basis in sequency order: W[s, j] = +-1/sqrt(B)
    with row s the Walsh function of s sign changes (first entry positive).

    Built from Sylvester's natural-order Hadamard matrix H[k, j] =
    (-1)^popcount(k & j) by sorting its rows by their number of sign changes,
    so that the zigzag scan runs from low to high sequency as it runs from low
    to high frequency for the DCT.
    """
    B = int(block)
    if B < 1 or B & (B - 1):
        raise ValueError("Walsh-Hadamard order must be a power of two")
    H = np.array([[(-1.0) ** bin(k & j).count("1") for j in range(B)] for k in range(B)])
    changes = [int(np.count_nonzero(H[k, 1:] != H[k, :-1])) for k in range(B)]
    return H[np.argsort(changes, kind="stable")] / math.sqrt(B)


TRANSFORMS = ("dct", "wht")


def basis(block, transform="dct"):
    """The sensing transform's B x B basis: DCT-II (default) or Walsh-Hadamard."""
    if transform == "dct":
        return dct_matrix(block)
    if transform == "wht":
        return walsh_matrix(block)
    raise ValueError(f"unknown transform {transform!r}")


def zigzag(block):
    """JPEG zigzag scan of a B x B block as a list of (row, col) pairs.

    Anti-diagonal d = row + col runs 0 .. 2B-2.  On odd d the scan goes down
    the diagonal (row ascending), on even d up it (row descending), so the
    entry after DC is (0, 1): row = vertical frequency, col = horizontal.
    """
    B = int(block)
    order = []
    for d in range(2 * B - 1):
        rows = range(max(0, d - B + 1), min(d, B - 1) + 1)
        if d % 2 == 0:
            rows = reversed(list(rows))
        for r in rows:
            order.append((r, d - r))
    return order


def to_blocks(img, block):
    """(H', W') array -> (n_B, B, B) in raster block order."""
    B = int(block)
    Hc, Wc = img.shape[0] // B * B, img.shape[1] // B * B
    a = np.asarray(img[:Hc, :Wc], dtype=np.float64)
    return a.reshape(Hc // B, B, Wc // B, B).transpose(0, 2, 1, 3).reshape(-1, B, B)


def from_blocks(blocks, nby, nbx):
    """(n_B, B, B) -> (n_by B, n_bx B) image."""
    B = blocks.shape[1]
    return blocks.reshape(nby, nbx, B, B).transpose(0, 2, 1, 3).reshape(nby * B, nbx * B)


def block_dct(X, D):
    """C = D X D^T for each block of X (n_B, B, B), float64.

    Fixed order: T[r, v] = sum_j X[r, j] D[v, j] with j ascending, then
    C[u, v] = sum_r D[u, r] T[r, v] with r ascending; every product and every
    sum is rounded separately (numpy elementwise ops, no fused multiply-add).
    """
    X = np.asarray(X, dtype=np.float64)
    B = D.shape[0]
    T = np.zeros_like(X)
    for j in range(B):
        T = T + X[:, :, j:j + 1] * D[None, None, :, j]
    C = np.zeros_like(X)
    for r in range(B):
        C = C + D[None, :, r:r + 1] * T[:, r:r + 1, :]
    return C


def block_idct(C, D):
    """X = D^T C D for each block of C (n_B, B, B), float64.

    P[u, j] = sum_v C[u, v] D[v, j]; X[i, j] = sum_u D[u, i] P[u, j].
    """
    C = np.asarray(C, dtype=np.float64)
    B = D.shape[0]
    P = np.zeros_like(C)
    for v in range(B):
        P = P + C[:, :, v:v + 1] * D[None, None, v, :]
    X = np.zeros_like(C)
    for u in range(B):
        X = X + D[None, u, :, None] * P[:, u:u + 1, :]
    return X


# ---------------------------------------------------------------------------
# Phase-1 statistics
# ---------------------------------------------------------------------------

def bbv_stat(img, block, L, X0, nS):
    """BBV_i of every block (eq 19), exact integers, raster block order.

    For the block with top-left pixel (r0, c0) and k_j = X0 + j L:
      h = sum_j |I[r0, c0 + k_j] - I[r0, c0 + k_j - 1]|      (top row)
      v = sum_j |I[r0 + k_j, c0] - I[r0 + k_j - 1, c0]|      (left column)
    BBV_i = h(block) + v(block) + h(block below) + v(block to the right),
    where a block in the last block row (column) uses its own bottom row
    (right column) in place of the missing neighbour.
    """
    B = int(block)
    I = np.asarray(img).astype(np.int64)
    Hc, Wc, nbx, nby, nB = geometry(I.shape[0], I.shape[1], B)
    ks = [X0 + j * L for j in range(nS)]

    def row_var(r, c0):
        return sum(abs(int(I[r, c0 + k]) - int(I[r, c0 + k - 1])) for k in ks)

    def col_var(c, r0):
        return sum(abs(int(I[r0 + k, c]) - int(I[r0 + k - 1, c])) for k in ks)

    out = np.zeros(nB, dtype=np.int64)
    for by in range(nby):
        for bx in range(nbx):
            r0, c0 = by * B, bx * B
            top = row_var(r0, c0)
            left = col_var(c0, r0)
            bottom = row_var(r0 + B, c0) if by + 1 < nby else row_var(r0 + B - 1, c0)
            right = col_var(c0 + B, r0) if bx + 1 < nbx else col_var(c0 + B - 1, r0)
            out[by * nbx + bx] = top + left + bottom + right
    return out


def bbv_sample_pairs(height, width, block, L, X0, nS):
    """The pixel pairs (a, b) of every BBV sample (eq 19), as flat indices into
    the cropped H' x W' image; the sample's value is I[a] - I[b] (a the later
    pixel along the border).  Order: for each block in raster order its n_S
    top-row then its n_S left-column samples; then the n_S bottom-row samples
    of each block of the last block row; then the n_S right-column samples of
    each block of the last block column (M_BBV pairs in all)."""
    B = int(block)
    Hc, Wc, nbx, nby, nB = geometry(height, width, B)
    ks = [X0 + j * L for j in range(nS)]
    a, b = [], []

    def row(r, c0):
        for k in ks:
            a.append(r * Wc + c0 + k)
            b.append(r * Wc + c0 + k - 1)

    def col(c, r0):
        for k in ks:
            a.append((r0 + k) * Wc + c)
            b.append((r0 + k - 1) * Wc + c)

    for by in range(nby):
        for bx in range(nbx):
            row(by * B, bx * B)
            col(bx * B, by * B)
    for bx in range(nbx):
        row((nby - 1) * B + B - 1, bx * B)
    for by in range(nby):
        col((nbx - 1) * B + B - 1, by * B)
    return np.array(a, dtype=np.int64), np.array(b, dtype=np.int64)


def bbv_samples(img, block, L, X0, nS):
    """Signed BBV samples I[a] - I[b] in the order of bbv_sample_pairs; their
    absolute values are the terms of eq 19, which the encoder measures anyway
    and may send as extra measurements (Section V-A)."""
    I = np.asarray(img).astype(np.int64)
    Hc, Wc, _, _, _ = geometry(I.shape[0], I.shape[1], block)
    flat = I[:Hc, :Wc].reshape(-1)
    a, b = bbv_sample_pairs(I.shape[0], I.shape[1], block, L, X0, nS)
    return flat[a] - flat[b]


def dd_stat(img, block, m1, T, transform="dct"):
    """n_i = #{z < m1 : |C_i[zigzag[z]]| > T}, C_i from block_dct (float64)
    with the sensing transform's basis."""
    B = int(block)
    D = basis(B, transform)
    C = block_dct(to_blocks(img, B), D)
    zz = zigzag(B)[:m1]
    if m1 == 0:
        return np.zeros(C.shape[0], dtype=np.int64)
    rows = np.array([p[0] for p in zz])
    cols = np.array([p[1] for p in zz])
    first = C[:, rows, cols]
    return np.count_nonzero(np.abs(first) > T, axis=1).astype(np.int64)


# ---------------------------------------------------------------------------
# Budget
# ---------------------------------------------------------------------------

def apportion(pool, weights, cap):
    """Split `pool` coefficients over blocks in proportion to `weights`.

    floor shares (eqs 22, 23); cap each block at `cap` and re-split what is
    left over the uncapped blocks; hand the final floor leftover to the
    largest remainders, ties to the lower index.  Exact integer arithmetic.
    Requires 0 <= pool <= cap * n.
    """
    w = np.asarray(weights, dtype=np.int64)
    n = w.shape[0]
    cap = int(cap)
    P = int(pool)
    if P < 0 or P > cap * n:
        raise DomainError("pool outside [0, cap * n_B]")
    a = np.zeros(n, dtype=np.int64)
    active = np.ones(n, dtype=bool) if cap > 0 else np.zeros(n, dtype=bool)
    while True:
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            return a
        wa = w[idx].copy()
        S = int(wa.sum())
        if S == 0:
            wa[:] = 1
            S = idx.size
        pw = P * wa
        q = pw // S
        over = q >= cap
        if over.any():
            hit = idx[over]
            a[hit] = cap
            P -= cap * hit.size
            active[hit] = False
            continue
        a[idx] = q
        R = P - int(q.sum())
        if R > 0:
            rem = pw - q * S
            order = np.lexsort((idx, -rem))
            a[idx[order[:R]]] += 1
        return a


def budget(img, block, subrate, method, transform="dct"):
    """Per-block coefficient counts k (int64, raster order) and the phase-1
    statistic (BBV_i or n_i; zeros for ZZ) for one image (Alg 1/2 steps 1-4).
    DD's phase-1 coefficients are those of the sensing transform."""
    s = budget_scalars(img.shape[0], img.shape[1], block, subrate, method)
    nB = s["nB"]
    if s["mode"] == ZZ:
        return np.full(nB, s["kz"], dtype=np.int64), np.zeros(nB, dtype=np.int64)
    if s["mode"] == BBV:
        w = bbv_stat(img, block, s["L"], s["X0"], s["nS"])
        return apportion(s["pool"], w, s["cap"]), w
    w = dd_stat(img, block, s["m1"], s["T"], transform)
    return s["m1"] + apportion(s["pool"], w, s["cap"]), w


def offsets(k):
    """Exclusive prefix sum: block i's coefficients are y[off[i] : off[i] + k[i]]."""
    k = np.asarray(k, dtype=np.int64)
    return np.concatenate([[0], np.cumsum(k)[:-1]]).astype(np.int64) if k.size else k


# ---------------------------------------------------------------------------
# Sensing and reconstruction (the block-diagonal operator of eq 26)
# ---------------------------------------------------------------------------

def _zigzag_index(block):
    B = int(block)
    zz = zigzag(B)
    return np.array([p[0] for p in zz]), np.array([p[1] for p in zz])


def sense_op(x_img, block, k, transform="dct"):
    """A x: for each block the first k_i zigzag transform coefficients, packed
    block after block (raster order), zigzag order within a block."""
    B = int(block)
    C = block_dct(to_blocks(x_img, B), basis(B, transform))
    rows, cols = _zigzag_index(B)
    czz = C[:, rows, cols]                       # (n_B, B^2) in zigzag order
    k = np.asarray(k, dtype=np.int64)
    keep = np.arange(B * B)[None, :] < k[:, None]
    return czz[keep]


def sense_adjoint(z, block, k, nby, nbx, transform="dct"):
    """A* z: put each block's coefficients back at their zigzag positions,
    zero elsewhere, and apply the inverse block transform."""
    B = int(block)
    rows, cols = _zigzag_index(B)
    k = np.asarray(k, dtype=np.int64)
    keep = np.arange(B * B)[None, :] < k[:, None]
    czz = np.zeros((k.size, B * B), dtype=np.float64)
    czz[keep] = np.asarray(z, dtype=np.float64)
    C = np.zeros((k.size, B, B), dtype=np.float64)
    C[:, rows, cols] = czz
    return from_blocks(block_idct(C, basis(B, transform)), nby, nbx)


def sense(img, block, k, transform="dct"):
    """Phase-2 measurement vector y (Alg 1 step 4, Alg 2 step 5): the first
    k_i zigzag 2D-transform coefficients of each block of the cropped image."""
    return sense_op(np.asarray(img, dtype=np.float64), block, k, transform)


def reconstruct(y, block, k, height, width, transform="dct"):
    """Real-time decoder output I_o: zero-filled masked inverse 2D transform."""
    _, _, nbx, nby, _ = geometry(height, width, block)
    return sense_adjoint(np.asarray(y, dtype=np.float64), block, k, nby, nbx, transform)


def encode(img, block, subrate, method, transform="dct"):
    """Budget + sensing for one image: returns (k, stat, y)."""
    k, stat = budget(img, block, subrate, method, transform)
    return k, stat, sense(img, block, k, transform)
