"""Explicit projection matrix W of exact ray-pixel intersection lengths (oracle).

Section 2.1 (eq. sys) defines W in R^{M x N} mapping the image onto the
projection data; the paper notes W is sparse with O(sqrt N) non-zeros per
column.  Here w_ij is the length of the intersection of ray i with the closed
square of pixel j, assembled explicitly, one angle block at a time:

  1. clip the ray's line to the image square;
  2. list the line parameters where it crosses every vertical grid line
     x = -1 + a h and every horizontal grid line y = -1 + b h;
  3. sort them; consecutive differences are segment lengths;
  4. each non-empty segment lies inside one pixel, found from its midpoint.

A ray parallel to an axis is handled by index: a line strictly inside a pixel
column (row) gives h to every pixel of it; a line lying on a grid line gives
h/2 to each of the (up to two) image pixels sharing that edge.  This is the
limit of the exact length as the angle tends to the axis, and keeps the
reflection and transpose symmetries of the geometry exact.

Parity status: pinned by row sums = chord lengths, disk chord lengths,
brute-force polygon clipping on tiny grids, and exact symmetries.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import Geometry, bin_offsets, direction


def _axis_block(n: int, nb: int, vertical: bool) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """COO triplets of an axis-parallel angle block.

    vertical=True: theta = 0, rays are lines x = s_j (they cross every row).
    vertical=False: theta = pi/2, rays are lines y = s_j.
    Position of line j measured in pixel edges from the left/bottom border:
    e_j = (2j - nb + 1 + n)/2, exact in integers via q = 2j - nb + 1 + n.
    """
    h = 2.0 / n
    rows, cols, vals = [], [], []
    lines = np.arange(n)
    for j in range(nb):
        q = 2 * j - nb + 1 + n          # 2 * e_j
        if q % 2 == 0:                  # on a grid line: share h/2
            a = q // 2
            targets = [(a - 1, 0.5 * h), (a, 0.5 * h)]
        else:                           # strictly inside column/row (q-1)/2
            targets = [((q - 1) // 2, h)]
        for idx, w in targets:
            if 0 <= idx < n:
                if vertical:
                    pix = lines * n + idx   # column idx, every row
                else:
                    pix = idx * n + lines   # row idx, every column
                rows.append(np.full(n, j, dtype=np.int64))
                cols.append(pix)
                vals.append(np.full(n, w))
    if not rows:
        return (np.zeros(0, np.int64),) * 2 + (np.zeros(0),)
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def _traverse(g: Geometry, c: float, s: float, t: np.ndarray):
    """Grid-crossing traversal of non-axis rays with offsets t -> COO (ray, pixel, length)."""
    n = g.n
    h = g.h
    grid = -1.0 + np.arange(n + 1) * h             # grid line coordinates
    # point on ray: x = t c - lam s, y = t s + lam c
    bx, by = t * c, t * s
    # slab clipping to the square
    ax0, ax1 = (bx - 1.0) / s, (bx + 1.0) / s      # x = -1 and x = +1
    ay0, ay1 = (-1.0 - by) / c, (1.0 - by) / c     # y = -1 and y = +1
    lo = np.maximum(np.minimum(ax0, ax1), np.minimum(ay0, ay1))
    hi = np.minimum(np.maximum(ax0, ax1), np.maximum(ay0, ay1))
    # crossing parameters of all grid lines
    lam_x = (bx[:, None] - grid[None, :]) / s      # x = grid
    lam_y = (grid[None, :] - by[:, None]) / c      # y = grid
    lam = np.concatenate([lam_x, lam_y, lo[:, None], hi[:, None]], axis=1)
    lam = np.minimum(np.maximum(lam, lo[:, None]), hi[:, None])
    lam.sort(axis=1)
    seg = np.diff(lam, axis=1)                     # lengths (direction is unit)
    mid = 0.5 * (lam[:, 1:] + lam[:, :-1])
    keep = seg > 1e-12 * h
    ray = np.broadcast_to(np.arange(len(t))[:, None], seg.shape)[keep]
    length = seg[keep]
    mid = mid[keep]
    xm = bx[ray] - mid * s
    ym = by[ray] + mid * c
    ix = np.clip(np.floor((xm + 1.0) / h).astype(np.int64), 0, n - 1)
    iy = np.clip(np.floor((ym + 1.0) / h).astype(np.int64), 0, n - 1)
    return ray, iy * n + ix, length


def angle_block(g: Geometry, k: int) -> sp.csr_matrix:
    """Rows k*nb .. k*nb+nb-1 of W as an (nb x N) CSR matrix (float64)."""
    c, s = direction(k, g.m)
    if s == 0.0 or c == 0.0:
        r, col, v = _axis_block(g.n, g.nb, vertical=(s == 0.0))
    else:
        r, col, v = _traverse(g, c, s, bin_offsets(g.nb, g.n))
    blk = sp.csr_matrix((v, (r, col)), shape=(g.nb, g.N))
    blk.sum_duplicates()
    return blk


def ray_rows(g: Geometry, k: int, bins) -> sp.csr_matrix:
    """Rows of W for angle k and the listed bins only (len(bins) x N)."""
    bins = np.asarray(bins, dtype=np.int64)
    c, s = direction(k, g.m)
    if s == 0.0 or c == 0.0:
        return angle_block(g, k)[bins]
    r, col, v = _traverse(g, c, s, bin_offsets(g.nb, g.n)[bins])
    blk = sp.csr_matrix((v, (r, col)), shape=(len(bins), g.N))
    blk.sum_duplicates()
    return blk


def clip_length(c, s, t, x0, x1, y0, y1):
    """Length of the line p.(c,s) = t inside the box [x0,x1] x [y0,y1] (vectorised).

    For non-axis lines only (c != 0 and s != 0); parametrisation as above.
    """
    bx, by = t * c, t * s
    a0, a1 = (bx - x0) / s, (bx - x1) / s
    b0, b1 = (y0 - by) / c, (y1 - by) / c
    lo = np.maximum(np.minimum(a0, a1), np.minimum(b0, b1))
    hi = np.minimum(np.maximum(a0, a1), np.maximum(b0, b1))
    return np.maximum(0.0, hi - lo)


def pixel_column(g: Geometry, pix: int) -> np.ndarray:
    """Column pix of W as a dense float64 vector of length M, by clipping every
    candidate ray to that one pixel square (axis rays by the index rule)."""
    n, nb, h = g.n, g.nb, g.h
    iy, ix = divmod(int(pix), n)
    x0, y0 = -1.0 + ix * h, -1.0 + iy * h
    xc, yc = x0 + 0.5 * h, y0 + 0.5 * h
    col = np.zeros(g.M)
    t_all = bin_offsets(nb, n)
    for k in range(g.m):
        c, s = direction(k, g.m)
        if s == 0.0 or c == 0.0:
            e = ix if s == 0.0 else iy            # pixel edges at 2e and 2e+2
            for j in range(nb):
                q = 2 * j - nb + 1 + n
                if 2 * e < q < 2 * e + 2:
                    col[k * nb + j] = h
                elif q == 2 * e or q == 2 * e + 2:
                    col[k * nb + j] = 0.5 * h
            continue
        tc = xc * c + yc * s
        js = np.nonzero(np.abs(t_all - tc) < h)[0]
        col[k * nb + js] = clip_length(c, s, t_all[js], x0, x0 + h, y0, y0 + h)
    return col


def system_matrix(g: Geometry, angles=None) -> sp.csr_matrix:
    """W (or the rows of the listed angles, stacked in that order) as CSR float64."""
    ks = range(g.m) if angles is None else angles
    return sp.vstack([angle_block(g, k) for k in ks], format="csr")


def project(W: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """b = W x for an image x [n][n] (float64)."""
    return W @ np.asarray(x, dtype=np.float64).ravel()


def backproject(W: sp.csr_matrix, y: np.ndarray) -> np.ndarray:
    """W^T y (float64, flat)."""
    return W.T @ np.asarray(y, dtype=np.float64).ravel()


def row_sums(W: sp.csr_matrix) -> np.ndarray:
    return np.asarray(W.sum(axis=1)).ravel()


def column_sums(W: sp.csr_matrix) -> np.ndarray:
    return np.asarray(W.sum(axis=0)).ravel()
