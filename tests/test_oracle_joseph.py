"""Pins of the Joseph-kernel oracle (Section 2.1 names Joseph's kernel for W).

- Images linear along the interpolation axis: Joseph's sum is the midpoint rule
  in the followed coordinate of a function that linear interpolation
  reproduces, so a ray that stays between the outermost pixel centres gets the
  exact line integral: the chord length 2/|cos a| times the value at the chord
  midpoint (closed form, no use of the assembly).
- Where the kernels coincide it equals the exact-length matrix (pinned on its
  own): at 45 degrees both footprints are the same triangle; at axis angles a
  ray through pixel centres gives h to each pixel it passes, and a ray on
  pixel edges h/2 to each neighbour.
- A planted mistake in the oracle (the interpolation anchored one pixel off)
  fails the linear pin.
"""
import numpy as np
import pytest

from oracle import joseph
from oracle.geometry import Geometry, bin_offsets, direction, pixel_centres
from oracle.projector import angle_block


@pytest.mark.parametrize("n,m,nb", [(16, 12, 23), (24, 18, 35), (9, 7, 13)])
def test_linear_images_give_exact_chord_integrals(n, m, nb):
    g = Geometry(n, m, nb)
    h = g.h
    xc = pixel_centres(n)
    rng = np.random.default_rng(n)
    t = bin_offsets(nb, n)
    checked = 0
    for k in range(m):
        c, s = direction(k, m)
        rows = abs(c) >= abs(s)
        a, b = (c, s) if rows else (s, c)
        alpha, beta = rng.normal(), rng.normal()
        # image linear in the interpolated coordinate (x when rows are followed)
        vals = alpha + beta * xc
        img = np.tile(vals, (n, 1)) if rows else np.tile(vals[:, None], (1, n))
        blk = joseph.joseph_block(g, k)
        sums = blk @ img.ravel()
        # rays whose crossing points stay within the outermost centres on every
        # followed line: |t/a| + |b/a| (1 - h/2) <= 1 - h/2
        lim = 1.0 - 0.5 * h
        ok = np.abs(t / a) + abs(b / a) * lim <= lim + 1e-12
        want = (2.0 / abs(a)) * (alpha + beta * t / a)
        assert np.allclose(sums[ok], want[ok], rtol=1e-12, atol=1e-12), k
        checked += int(ok.sum())
    assert checked > m


@pytest.mark.parametrize("n,nb", [(8, 12), (12, 17), (10, 15)])
def test_equals_exact_lengths_at_45_degrees(n, nb):
    g = Geometry(n, 4, nb)            # angles 0, 45, 90, 135 degrees
    for k in (1, 3):
        J = joseph.joseph_block(g, k).toarray()
        E = angle_block(g, k).toarray()
        assert np.allclose(J, E, rtol=0, atol=1e-14 * g.h), k


@pytest.mark.parametrize("n,nb", [(8, 8), (8, 9), (7, 7), (7, 8)])
def test_equals_exact_lengths_on_axis_rays(n, nb):
    """nb = n: bin centres on pixel centres; nb = n + 1: on pixel edges."""
    g = Geometry(n, 2, nb)            # 0 and 90 degrees
    for k in (0, 1):
        J = joseph.joseph_block(g, k).toarray()
        E = angle_block(g, k).toarray()
        assert np.allclose(J, E, rtol=0, atol=1e-14 * g.h), k


def test_weights_per_followed_line_sum_to_the_step():
    n, m, nb = 12, 10, 17
    g = Geometry(n, m, nb)
    for k in range(m):
        c, s = direction(k, m)
        rows = abs(c) >= abs(s)
        step = g.h / max(abs(c), abs(s))
        blk = joseph.joseph_block(g, k).toarray().reshape(nb, n, n)   # [ray][iy][ix]
        per_line = blk.sum(axis=2) if rows else blk.sum(axis=1)
        # lines where both interpolation pixels lie inside the image carry the full step
        full = np.isclose(per_line, step, rtol=1e-12)
        partial = per_line < step * (1 - 1e-12)
        assert np.all(full | partial)
        assert full.sum() > n


def test_misplaced_interpolation_fails_the_linear_pin(monkeypatch):
    """A planted mistake in the oracle (interpolation anchored one pixel off) is caught."""
    n, m, nb = 16, 12, 23
    g = Geometry(n, m, nb)
    k = 2
    c, s = direction(k, m)
    orig_floor = np.floor

    def shifted_floor(x):   # anchors the interpolation at floor(P) + 1
        return orig_floor(x) + 1.0

    monkeypatch.setattr(joseph.np, "floor", shifted_floor)
    blk = joseph.joseph_block(g, k)
    monkeypatch.undo()
    xc = pixel_centres(n)
    img = np.tile(0.5 + 2.0 * xc, (n, 1))
    t = bin_offsets(nb, n)
    want = (2.0 / abs(c)) * (0.5 + 2.0 * t / c)
    lim = 1.0 - 0.5 * g.h
    ok = np.abs(t / c) + abs(s / c) * lim <= lim
    assert not np.allclose((blk @ img.ravel())[ok], want[ok], rtol=1e-6)


def _kernel_form(g, joseph_coefficients):
    """W from the projectors' weight form, pixel driven: for pixel centre bin
    coordinate J (f = J - floor J) the bins floor J and floor J + 1 weigh
    clamp(C0 - f B) and clamp(C1 + f B) in [0, 1/u] (units of h), with
    B = 1/(u v), C0 = 1/(2u) + u B / 2, C1 = 1/(2u) + (u/2 - 1) B; exact
    lengths take v = min(|cos|, |sin|), Joseph's kernel v = u (reading D30)."""
    n, m, nb = g.n, g.m, g.nb
    hc, hb = 0.5 * (n - 1), 0.5 * (nb - 1)
    W = np.zeros((g.M, g.N))
    iy, ix = np.divmod(np.arange(g.N), n)
    for k in range(m):
        c, s = direction(k, m)
        u = max(abs(c), abs(s))
        v = u if joseph_coefficients else min(abs(c), abs(s))
        if v == 0.0:
            continue
        B = 1.0 / (u * v)
        C0 = 0.5 / u + 0.5 * u * B
        C1 = 0.5 / u + (0.5 * u - 1.0) * B
        Jc = (ix - hc) * c + (iy - hc) * s + hb
        j0 = np.floor(Jc)
        f = Jc - j0
        for j, w in ((j0, np.clip(C0 - f * B, 0.0, 1.0 / u)), (j0 + 1, np.clip(C1 + f * B, 0.0, 1.0 / u))):
            ok = (j >= 0) & (j < nb) & (w > 0)
            W[k * nb + j[ok].astype(int), np.arange(g.N)[ok]] += w[ok] * g.h
    return W


@pytest.mark.parametrize("n,m,nb", [(24, 18, 35), (16, 7, 23), (9, 10, 13)])
def test_kernel_weight_form_with_v_equal_u_is_joseph(n, m, nb):
    """Reading D30: the weight coefficients of the exact-length kernels with v replaced by u
    give Joseph's kernel (angles off the axes; the kernels treat v = 0 with a finite slope)."""
    g = Geometry(n, m, nb)
    J = joseph.joseph_matrix(g).toarray()
    K = _kernel_form(g, True)
    rows = np.concatenate([np.arange(k * nb, (k + 1) * nb) for k in range(m)
                           if min(abs(c) for c in direction(k, m)) > 0])
    assert np.abs(K[rows] - J[rows]).max() <= 1e-13 * g.h
    # and with v = min(|cos|, |sin|) the same form is the exact-length matrix
    E = angle_block_stack(g)
    Ke = _kernel_form(g, False)
    assert np.abs(Ke[rows] - E[rows]).max() <= 1e-12 * g.h


def angle_block_stack(g):
    return np.vstack([angle_block(g, k).toarray() for k in range(g.m)])


@pytest.mark.parametrize("n,m,nb", [(24, 18, 35), (16, 7, 23)])
def test_forward_weight_form_with_v_equal_u_is_joseph(n, m, nb):
    """The forward projector's per-row form w0 = clamp((1/2 - f) B + C, 0, 1/u),
    w1 = 1/u - w0 with B = 1/u, C = 1/(2u) (reading D30) is Joseph's interpolation:
    ray sums of random images agree with the oracle."""
    g = Geometry(n, m, nb)
    rng = np.random.default_rng(7)
    x = rng.random(g.N)
    J = joseph.joseph_matrix(g)
    hc, hb = 0.5 * (n - 1), 0.5 * (nb - 1)
    img = x.reshape(n, n)
    for k in range(m):
        c, s = direction(k, m)
        rows = abs(c) >= abs(s)
        a, b = (c, s) if rows else (s, c)
        u = abs(a)
        B, C = 1.0 / u, 0.5 / u
        got = np.zeros(nb)
        for j in range(nb):
            for r in range(n):
                P = hc + ((j - hb) - (r - hc) * b) / a
                i0 = int(np.floor(P))
                f = P - i0
                w0 = min(max((0.5 - f) * B + C, 0.0), 1.0 / u)
                for i, w in ((i0, w0), (i0 + 1, 1.0 / u - w0)):
                    if 0 <= i < n:
                        got[j] += w * g.h * (img[r, i] if rows else img[i, r])
        want = (J @ x)[k * nb:(k + 1) * nb]
        assert np.allclose(got, want, rtol=1e-12, atol=1e-14), k
