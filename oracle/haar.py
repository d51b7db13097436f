"""Haar intergrid operators and the full Haar packet transform H_L (oracle).

Definitions followed:
  * eq. intops: I_{h,1D}^{2h} (n/2 x n) has rows (1, 1)/sqrt(2) on consecutive
    pixel pairs; interpolation is its transpose.
  * eq. intops_wav: J_{h,1D}^{2h} has rows (1, -1)/sqrt(2) on the same pairs.
  * eq. 1of4 - 4of4: the 2D operators are Kronecker products
        LL = I (x) I,  LH = I (x) J,  HL = J (x) I,  HH = J (x) J
    acting on the row-major image vector (index iy*n + ix), so the left factor
    acts along y (rows) and the right factor along x (columns).
  * Section 3.1.3: a WMG cycle with ell levels splits the fine problem into
    4^(ell-1) subproblems of N/4^(ell-1) unknowns.  The transform here splits
    *every* subband again at each level (the full packet tree), L = ell - 1
    times.

Coefficient layout ("quadrant layout"): one level maps an s x s block to four
s/2 x s/2 quadrants [[LL, LH], [HL, HH]] (top-left LL, top-right LH, bottom-left
HL, bottom-right HH, "top" meaning smaller row index); the next level applies
the same step inside each quadrant.

Parity status: pinned by orthogonality of [I; J], perfect reconstruction,
the constant-image case, and brute-force comparison of the recursive transform
with an explicit dense Kronecker construction on small grids.
"""
from __future__ import annotations

import functools
import math

import numpy as np
import scipy.sparse as sp

SQRT1_2 = 1.0 / math.sqrt(2.0)


@functools.lru_cache(maxsize=None)
def intergrid_1d(n: int) -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """(I_{h,1D}^{2h}, J_{h,1D}^{2h}), each n/2 x n (eq. intops, eq. intops_wav)."""
    assert n % 2 == 0
    r = np.repeat(np.arange(n // 2), 2)
    c = np.arange(n)
    I = sp.csr_matrix((np.full(n, SQRT1_2), (r, c)), shape=(n // 2, n))
    sgn = np.tile([1.0, -1.0], n // 2)
    J = sp.csr_matrix((sgn * SQRT1_2, (r, c)), shape=(n // 2, n))
    return I, J


@functools.lru_cache(maxsize=None)
def step_operators_2d(n: int) -> dict[str, sp.csr_matrix]:
    """The four (N/4 x N) restriction operators of eq. 1of4 - 4of4 for an n x n grid."""
    I, J = intergrid_1d(n)
    return {
        "LL": sp.kron(I, I, format="csr"),
        "LH": sp.kron(I, J, format="csr"),
        "HL": sp.kron(J, I, format="csr"),
        "HH": sp.kron(J, J, format="csr"),
    }


_QUAD = {"LL": (0, 0), "LH": (0, 1), "HL": (1, 0), "HH": (1, 1)}


def haar_step(block: np.ndarray) -> np.ndarray:
    """One 2D Haar step on an s x s block -> s x s array of quadrants."""
    s = block.shape[0]
    ops = step_operators_2d(s)
    v = block.ravel()
    out = np.empty_like(block, dtype=np.float64)
    h = s // 2
    for name, (qr, qc) in _QUAD.items():
        out[qr * h:(qr + 1) * h, qc * h:(qc + 1) * h] = (ops[name] @ v).reshape(h, h)
    return out


def haar_step_adjoint(coef: np.ndarray) -> np.ndarray:
    """Transpose of haar_step (interpolation I_{2h,id}^h = (I_{h,id}^{2h})^T summed)."""
    s = coef.shape[0]
    ops = step_operators_2d(s)
    h = s // 2
    v = np.zeros(s * s)
    for name, (qr, qc) in _QUAD.items():
        v += ops[name].T @ coef[qr * h:(qr + 1) * h, qc * h:(qc + 1) * h].ravel()
    return v.reshape(s, s)


def packet_transform(x: np.ndarray, L: int) -> np.ndarray:
    """H_L x: L levels of the 2D step, each applied to every subband (quadrant layout)."""
    a = np.array(x, dtype=np.float64).reshape(int(math.isqrt(np.size(x))), -1)
    n = a.shape[0]
    for lev in range(L):
        s = n >> lev
        for r0 in range(0, n, s):
            for c0 in range(0, n, s):
                a[r0:r0 + s, c0:c0 + s] = haar_step(a[r0:r0 + s, c0:c0 + s])
    return a


def packet_adjoint(c: np.ndarray, L: int) -> np.ndarray:
    """H_L^T c, undoing the levels in reverse order."""
    a = np.array(c, dtype=np.float64).reshape(int(math.isqrt(np.size(c))), -1)
    n = a.shape[0]
    for lev in reversed(range(L)):
        s = n >> lev
        for r0 in range(0, n, s):
            for c0 in range(0, n, s):
                a[r0:r0 + s, c0:c0 + s] = haar_step_adjoint(a[r0:r0 + s, c0:c0 + s])
    return a


def _block_level_matrix(n: int, s: int) -> sp.csr_matrix:
    """N x N sparse matrix applying haar_step to every s x s block of an n x n array."""
    ops = step_operators_2d(s)
    h = s // 2
    rows, cols, vals = [], [], []
    loc = np.arange(s * s).reshape(s, s)
    for r0 in range(0, n, s):
        for c0 in range(0, n, s):
            gidx = ((r0 + np.arange(s))[:, None] * n + (c0 + np.arange(s))[None, :])
            for name, (qr, qc) in _QUAD.items():
                op = ops[name].tocoo()
                out_loc = loc[qr * h:(qr + 1) * h, qc * h:(qc + 1) * h].ravel()
                rows.append(gidx.ravel()[out_loc[op.row]])
                cols.append(gidx.ravel()[op.col])
                vals.append(op.data)
    N = n * n
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


@functools.lru_cache(maxsize=8)
def packet_matrix(n: int, L: int) -> sp.csr_matrix:
    """H_L as an explicit N x N sparse matrix (rows in quadrant layout)."""
    H = sp.identity(n * n, format="csr")
    for lev in range(L):
        H = _block_level_matrix(n, n >> lev) @ H
    H = H.tocsr()
    H.eliminate_zeros()
    return H


def subband_of(row: int, col: int, n: int, L: int) -> tuple[int, int]:
    """(packet index p in 0..4^L-1, coarse-grid index J) of a quadrant-layout position.

    The coarse grid after L levels has side n/2^L; position (row, col) lies in
    sub-block (row // (n/2^L), col // (n/2^L)) which identifies the packet.
    """
    cs = n >> L
    p = (row // cs) * (1 << L) + (col // cs)
    J = (row % cs) * cs + (col % cs)
    return p, J
