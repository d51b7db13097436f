"""Explicit projection matrix of Joseph's interpolation kernel (oracle; test
infrastructure only: only tests, the smoke check and the benchmark's CPU
baseline use this package).

Section 2.1 names Joseph's kernel for W.  Its definition, restated: a ray is
followed along the image axis closest to its own direction.  On the centre
line of every image row (or column) it crosses, the image value at the
crossing point is the linear interpolation between the two nearest pixel
centres of that row (column); pixels outside the image count as zero.  The
ray integral is the sum of these values, each times the length of the ray
between consecutive centre lines, h / |cos a| with a the angle between the ray
and the axis followed.

Same geometry as the exact-length oracle: ray (k, j) is the line
p.(c, s) = t_j (theta_k = k pi / m, t_j = (j - (nb-1)/2) h); pixel (ix, iy),
index iy n + ix, has centre (-1 + (ix + 1/2) h, -1 + (iy + 1/2) h).  For
|c| >= |s| the ray direction (-s, c) is closer to the y axis and the rows iy
are followed (interpolation along x); otherwise the columns ix.

Parity status: pinned in tests by exactness for images linear along the
interpolation axis (closed-form ray sums), equality with the exact-length
matrix where the two kernels coincide (45 degrees, and axis rays through pixel
centres or on pixel edges), and the per-row weight sum h / |cos a|.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import Geometry, direction


def joseph_block(g: Geometry, k: int) -> sp.csr_matrix:
    """Rows k*nb .. k*nb+nb-1 of Joseph's W as an (nb x N) CSR matrix (float64)."""
    n, nb, h = g.n, g.nb, g.h
    c, s = direction(k, g.m)
    rows_follow = abs(c) >= abs(s)
    a, b = (c, s) if rows_follow else (s, c)   # p.(c, s) = t solved for the interpolated coordinate
    step = h / abs(a)
    # crossing point of ray j with centre line r in pixel index units: with
    # t_j = (j - hb) h and the line at (r - hc) h, the point (t_j - y_r b) / a
    # is at index hc + ((j - hb) - (r - hc) b) / a (exact for axis rays)
    hc, hb = 0.5 * (n - 1), 0.5 * (nb - 1)
    tj = np.arange(nb, dtype=np.float64) - hb
    yr = np.arange(n, dtype=np.float64) - hc
    P = hc + (tj[:, None] - yr[None, :] * b) / a
    i0 = np.floor(P)
    f = P - i0
    i0 = i0.astype(np.int64)
    ray = np.broadcast_to(np.arange(nb)[:, None], P.shape)
    line = np.broadcast_to(np.arange(n)[None, :], P.shape)
    r_all, c_all, v_all = [], [], []
    for idx, w in ((i0, 1.0 - f), (i0 + 1, f)):
        keep = (idx >= 0) & (idx < n) & (w > 0.0)
        ii, ll = idx[keep], line[keep]
        pix = ll * n + ii if rows_follow else ii * n + ll
        r_all.append(ray[keep])
        c_all.append(pix)
        v_all.append(w[keep] * step)
    blk = sp.csr_matrix((np.concatenate(v_all), (np.concatenate(r_all), np.concatenate(c_all))),
                        shape=(nb, g.N))
    blk.sum_duplicates()
    return blk


def joseph_matrix(g: Geometry, angles=None) -> sp.csr_matrix:
    """Joseph's W (or the rows of the listed angles, stacked in that order) as CSR float64."""
    ks = range(g.m) if angles is None else angles
    return sp.vstack([joseph_block(g, k) for k in ks], format="csr")
