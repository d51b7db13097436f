"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random numbers and rasterises ellipses. It holds none of the
reconstruction method's arithmetic (no projection, no wavelet, no solver), so
both the CPU oracle and the HIP path can consume its outputs without sharing
any code with each other.

Conventions (the image domain of the workloads):
  * the image covers [-1, 1]^2 on an n x n grid with pixel size h = 2/n;
  * pixel (ix, iy) has centre (-1 + (ix + 1/2) h, -1 + (iy + 1/2) h) and is
    stored row-major at index iy * n + ix (y grows with iy).

The paper's test object is a "Shepp-Logan type" phantom whose parameters it
does not print (Section 4.1); seeded sums of random ellipses stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng",
    "ellipse_params",
    "ellipse_phantom",
    "standard_normal",
    "default_bins",
    "default_levels",
    "batch_mix",
    "serving_mix",
    "WORKLOADS",
]


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for a seed."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def ellipse_params(n_ellipses: int, gen: np.random.Generator) -> np.ndarray:
    """Draw ellipse parameters, one row per ellipse.

    Columns: centre x, centre y, semi-axis a, semi-axis b, rotation, intensity.
    Per ellipse, in this order: centre radius 0.8*sqrt(U), centre angle 2*pi*U,
    a ~ U[0.05, 0.4], b ~ U[0.05, 0.4], rotation ~ U[0, pi), intensity ~ U[0.1, 1].
    """
    out = np.empty((n_ellipses, 6), dtype=np.float64)
    for e in range(n_ellipses):
        r = 0.8 * math.sqrt(gen.random())
        phi = 2.0 * math.pi * gen.random()
        a = gen.uniform(0.05, 0.4)
        b = gen.uniform(0.05, 0.4)
        rot = gen.uniform(0.0, math.pi)
        val = gen.uniform(0.1, 1.0)
        out[e] = (r * math.cos(phi), r * math.sin(phi), a, b, rot, val)
    return out


def ellipse_phantom(n: int, n_ellipses: int, seed: int) -> np.ndarray:
    """Pixel-centre sampled sum of random ellipses on [-1,1]^2, float64 [n][n].

    Each ellipse is evaluated only on the pixels inside the square that bounds
    its circumscribed circle (radius max(a, b)); pixels outside that square
    are outside the ellipse, so the sum equals the one over the whole grid.
    """
    params = ellipse_params(n_ellipses, rng(seed))
    h = 2.0 / n
    c = -1.0 + (np.arange(n) + 0.5) * h
    img = np.zeros((n, n), dtype=np.float64)
    for cx, cy, a, b, rot, val in params:
        rad = max(a, b)
        ix0 = max(0, int(math.floor((cx - rad + 1.0) / h)) - 1)
        ix1 = min(n, int(math.ceil((cx + rad + 1.0) / h)) + 1)
        iy0 = max(0, int(math.floor((cy - rad + 1.0) / h)) - 1)
        iy1 = min(n, int(math.ceil((cy + rad + 1.0) / h)) + 1)
        if ix0 >= ix1 or iy0 >= iy1:
            continue
        dx = c[None, ix0:ix1] - cx        # [1, w]
        dy = c[iy0:iy1, None] - cy        # [h, 1]
        ca, sa = math.cos(rot), math.sin(rot)
        u = (dx * ca + dy * sa) / a
        v = (-dx * sa + dy * ca) / b
        img[iy0:iy1, ix0:ix1] += val * ((u * u + v * v) <= 1.0)
    return img


def _ellipse_phantom_full_grid(n: int, n_ellipses: int, seed: int) -> np.ndarray:
    """The same phantom evaluated on every pixel for every ellipse (slow; tests)."""
    params = ellipse_params(n_ellipses, rng(seed))
    h = 2.0 / n
    c = -1.0 + (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")  # X[iy, ix], Y[iy, ix]
    img = np.zeros((n, n), dtype=np.float64)
    for cx, cy, a, b, rot, val in params:
        dx = X - cx
        dy = Y - cy
        ca, sa = math.cos(rot), math.sin(rot)
        u = (dx * ca + dy * sa) / a
        v = (-dx * sa + dy * ca) / b
        img += val * ((u * u + v * v) <= 1.0)
    return img


def standard_normal(size: int, seed: int) -> np.ndarray:
    """N(0,1) draws (float64) for additive noise; callers scale them."""
    return rng(seed).standard_normal(size)


def uniform_noise(size: int, seed: int) -> np.ndarray:
    """U(-1, 1) draws (float64) for the paper's white-noise model
    eps = alpha U(-1, 1) max|b| (Section 4.3, eq. noise_term); callers scale them."""
    return rng(seed).uniform(-1.0, 1.0, size)


def default_bins(side: int) -> int:
    """Detector bins of width one pixel covering the image diagonal."""
    return int(math.ceil(side * math.sqrt(2.0)))


def default_levels(side: int) -> int:
    """Number of multigrid levels for a side: coarsest subproblem side min(128, side/2)."""
    return max(2, int(round(math.log2(side))) - 6)


@dataclass(frozen=True)
class Request:
    """One reconstruction request of a batched or served workload."""

    index: int
    side: int
    n_angles: int
    n_bins: int
    n_ellipses: int
    tol: float
    noise: float
    seed: int
    arrival_s: float = 0.0


def batch_mix(count: int = 256, seed: int = 3000) -> list[Request]:
    """Batched workload: side in {128,256,512,1024}, angles in {90,180,360,720}."""
    g = rng(seed)
    out = []
    for i in range(count):
        side = int(g.choice([128, 256, 512, 1024]))
        ang = int(g.choice([90, 180, 360, 720]))
        ne = int(g.integers(5, 31))
        out.append(Request(i, side, ang, default_bins(side), ne, 1e-3, 0.01, seed + i))
    return out


def serving_mix(count: int, rate_hz: float, seed: int = 4000) -> list[Request]:
    """Served workload with Poisson arrivals at ``rate_hz``.

    Side from {256: 40%, 512: 30%, 1024: 20%, 2048: 10%}; angles uniform in
    side/2 .. 1.5*side; tolerance from {1e-2, 1e-3}; 1% noise.
    """
    g = rng(seed)
    sides = np.array([256, 512, 1024, 2048])
    probs = np.array([0.4, 0.3, 0.2, 0.1])
    t = 0.0
    out = []
    for i in range(count):
        t += g.exponential(1.0 / rate_hz)
        side = int(g.choice(sides, p=probs))
        ang = int(g.integers(side // 2, (3 * side) // 2 + 1))
        tol = float(g.choice([1e-2, 1e-3]))
        ne = int(g.integers(5, 31))
        out.append(Request(i, side, ang, default_bins(side), ne, tol, 0.01, seed + i, t))
    return out


# The five workload shapes: (side, angles, bins, levels, ellipses, noise fraction)
WORKLOADS = {
    "tiny64_f64": dict(n=64, m=90, nb=64, levels=2, ellipses=10, noise=0.0, seed=0),
    "ct512": dict(n=512, m=360, nb=725, levels=3, ellipses=20, noise=0.01, seed=1000),
    "ct2048": dict(n=2048, m=2048, nb=2897, levels=5, ellipses=40, noise=0.005, seed=2000),
}
