"""Pins of the oracle projection matrix W against geometry it must reproduce.

  * row sums equal the chord length of the ray through [-1,1]^2 (closed form);
  * every entry equals an independent edge-intersection computation on tiny grids;
  * a pixelised disk projects to 2 sqrt(r^2 - d^2) up to O(h), first order in h;
  * reflection x -> -x and transpose x <-> y map the sinogram exactly as the
    angle set predicts;
  * axis-parallel rays carry exactly h or h/2;
  * nnz(W) is close to (4/pi) m n^2 (mean chord count of a line through a pixel grid).
"""
import math

import numpy as np
import pytest

from oracle.geometry import Geometry, bin_offsets, chord_through_square, direction
from oracle.projector import (angle_block, backproject, pixel_column, project, ray_rows,
                              row_sums, system_matrix)

SMALL = [(8, 12, 12), (16, 7, 23), (16, 20, 16), (32, 45, 46), (12, 4, 17)]


@pytest.mark.parametrize("n,m,nb", SMALL)
def test_row_sums_are_chord_lengths(n, m, nb):
    g = Geometry(n, m, nb)
    rs = row_sums(system_matrix(g))
    for k in range(m):
        c, s = direction(k, m)
        for j, t in enumerate(bin_offsets(nb, n)):
            want = chord_through_square(c, s, t)
            if (s == 0.0 or c == 0.0) and abs(abs(t) - 1.0) < 1e-12:
                want = 1.0  # boundary-tangent axis ray: h/2 on each of n pixels
            assert abs(rs[k * nb + j] - want) < 1e-13, (k, j)


def _edge_chord(c, s, t, x0, x1, y0, y1):
    """Chord of a line inside an axis box from its intersections with the 4 edges."""
    pts = []
    # edges x = x0, x = x1 (vertical): solve y from c x + s y = t
    for xe in (x0, x1):
        if s != 0.0:
            y = (t - c * xe) / s
            if y0 - 1e-15 <= y <= y1 + 1e-15:
                pts.append((xe, y))
    for ye in (y0, y1):
        if c != 0.0:
            x = (t - s * ye) / c
            if x0 - 1e-15 <= x <= x1 + 1e-15:
                pts.append((x, ye))
    best = 0.0
    for a in pts:
        for b in pts:
            best = max(best, math.hypot(a[0] - b[0], a[1] - b[1]))
    return best


@pytest.mark.parametrize("n,m,nb", [(6, 9, 9), (8, 10, 12), (5, 7, 8)])
def test_entries_match_edge_intersections(n, m, nb):
    g = Geometry(n, m, nb)
    W = system_matrix(g).toarray()
    h = g.h
    for k in range(m):
        c, s = direction(k, m)
        if c == 0.0 or s == 0.0:
            continue
        for j, t in enumerate(bin_offsets(nb, n)):
            for iy in range(n):
                for ix in range(n):
                    x0, y0 = -1 + ix * h, -1 + iy * h
                    want = _edge_chord(c, s, t, x0, x0 + h, y0, y0 + h)
                    assert abs(W[k * nb + j, iy * n + ix] - want) < 1e-13


@pytest.mark.parametrize("n,m,nb", [(8, 12, 12), (16, 20, 16), (10, 6, 15)])
def test_axis_rays_weights(n, m, nb):
    g = Geometry(n, m, nb)
    h = g.h
    for k in (0, m // 2) if m % 2 == 0 else (0,):
        blk = angle_block(g, k).toarray()
        vals = np.unique(np.round(blk[blk != 0] / h, 15))
        assert set(vals) <= {0.5, 1.0}
        # every row carries its full share: n*h, or n*h/2 when tangent to the border
        rs = blk.sum(axis=1)
        for j, t in enumerate(bin_offsets(nb, n)):
            if abs(t) < 1 - 1e-12:
                assert abs(rs[j] - 2.0) < 1e-13
            elif abs(abs(t) - 1) < 1e-12:
                assert abs(rs[j] - 1.0) < 1e-13
            else:
                assert rs[j] == 0.0


def _disk(n, r, cx, cy):
    h = 2.0 / n
    cc = -1 + (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(cc, cc, indexing="xy")
    return ((X - cx) ** 2 + (Y - cy) ** 2 <= r * r).astype(float)


def test_disk_chords_first_order():
    r, cx, cy = 0.5, 0.13, -0.21
    errs = []
    for n in (32, 64, 128):
        m, nb = 24, int(math.ceil(n * math.sqrt(2)))
        g = Geometry(n, m, nb)
        b = project(system_matrix(g), _disk(n, r, cx, cy))
        want = np.zeros(g.M)
        for k in range(m):
            c, s = direction(k, m)
            d = bin_offsets(nb, n) - (cx * c + cy * s)
            want[k * nb:(k + 1) * nb] = 2 * np.sqrt(np.maximum(r * r - d * d, 0.0))
        errs.append(np.linalg.norm(b - want) / np.linalg.norm(want))
    # pixelisation error is first order in h: relative L2 error halves per refinement
    assert errs[0] < 0.06
    assert errs[1] < errs[0] / 1.7 and errs[2] < errs[1] / 1.6


@pytest.mark.parametrize("n,m,nb", [(16, 20, 23), (16, 12, 16), (12, 8, 17)])
def test_reflection_and_transpose_symmetry(n, m, nb):
    g = Geometry(n, m, nb)
    W = system_matrix(g)
    x = np.random.default_rng(5).random((n, n))
    b = project(W, x).reshape(m, nb)
    bf = project(W, x[:, ::-1]).reshape(m, nb)    # x -> -x
    for k in range(m):
        want = b[m - k] if k >= 1 else b[0, ::-1]
        assert np.allclose(bf[k], want, atol=1e-13, rtol=0)
    bt = project(W, x.T).reshape(m, nb)           # x <-> y
    for k in range(m):
        if 2 * k <= m:
            want = b[m // 2 - k]
        else:
            want = b[3 * m // 2 - k, ::-1]
        assert np.allclose(bt[k], want, atol=1e-13, rtol=0)


def test_nnz_close_to_mean_chord_count():
    for n, m in ((64, 90), (128, 60)):
        nb = int(math.ceil(n * math.sqrt(2)))
        nnz = system_matrix(Geometry(n, m, nb)).nnz
        assert abs(nnz / (4 / math.pi * m * n * n) - 1) < 0.03


def test_adjoint_identity():
    g = Geometry(32, 30, 46)
    W = system_matrix(g)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(g.N), rng.standard_normal(g.M)
    lhs = project(W, x) @ y
    rhs = x @ backproject(W, y)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_sampled_rows_and_columns_match_full_matrix():
    g = Geometry(24, 18, 35)
    W = system_matrix(g).toarray()
    for k in (0, 3, 9, 17):
        bins = [0, 5, 17, 34]
        got = ray_rows(g, k, bins).toarray()
        assert np.allclose(got, W[[k * g.nb + j for j in bins]], atol=1e-14, rtol=0)
    for pix in (0, 23, 24 * 11 + 7, 24 * 24 - 1):
        assert np.allclose(pixel_column(g, pix), W[:, pix], atol=1e-14, rtol=0)
