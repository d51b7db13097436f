"""Geometry conventions of the 2D parallel-beam problem (oracle side).

Section 2.1 (eq. sys) states the problem W x = b with x an n x n image and b
holding m angles times the detector beams.  The paper leaves the coordinates
unstated; this module fixes the readings used throughout:

  * image domain [-1, 1]^2, pixel size h = 2/n, pixel (ix, iy) centred at
    (-1 + (ix+1/2) h, -1 + (iy+1/2) h), flat index iy*n + ix;
  * m equiangular directions over 180 degrees (Section 4.1): theta_k = k*pi/m;
  * ray (k, j) is the line {p : p . (cos theta_k, sin theta_k) = s_j} with
    s_j = (j - (nb-1)/2) * h, one line per detector bin of width one pixel;
  * sinogram flat index k*nb + j.

At k = 0 and 2k = m the direction is snapped to the axis by index, because
cos(pi/2) is not zero in floating point.

Parity status: pinned through the projector tests (row sums, symmetries).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Geometry:
    n: int        # image side in pixels
    m: int        # number of projection angles
    nb: int       # detector bins per angle

    @property
    def h(self) -> float:
        return 2.0 / self.n

    @property
    def N(self) -> int:
        return self.n * self.n

    @property
    def M(self) -> int:
        return self.m * self.nb


def direction(k: int, m: int) -> tuple[float, float]:
    """(cos theta_k, sin theta_k) with theta_k = k*pi/m, axis angles snapped by index."""
    if k == 0:
        return 1.0, 0.0
    if 2 * k == m:
        return 0.0, 1.0
    t = k * math.pi / m
    return math.cos(t), math.sin(t)


def directions(m: int) -> np.ndarray:
    return np.array([direction(k, m) for k in range(m)], dtype=np.float64)


def bin_offsets(nb: int, n: int) -> np.ndarray:
    """Signed distance s_j of each ray from the origin."""
    return (np.arange(nb, dtype=np.float64) - (nb - 1) / 2.0) * (2.0 / n)


def pixel_centres(n: int) -> np.ndarray:
    return -1.0 + (np.arange(n, dtype=np.float64) + 0.5) * (2.0 / n)


def chord_through_square(c: float, s: float, t: float) -> float:
    """Length of the line p.(c,s) = t inside [-1,1]^2 (closed form of the clip).

    Used to pin row sums of W: a ray's weights add up to its chord length.
    """
    # Parametrise p = t*(c,s) + lam*(-s,c); intersect slabs |x|<=1, |y|<=1.
    lo, hi = -math.inf, math.inf
    for base, d in ((t * c, -s), (t * s, c)):
        if d == 0.0:
            if abs(base) > 1.0:
                return 0.0
            continue
        a, b = (-1.0 - base) / d, (1.0 - base) / d
        lo, hi = max(lo, min(a, b)), min(hi, max(a, b))
    return max(0.0, hi - lo)
