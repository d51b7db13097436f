"""GPU parity of the operators over a sweep of small geometries (through the C
ABI, against the CPU float64 oracle's W: exact intersection lengths and
Joseph's kernel).

Small images stress the forward projector's per-block set-up: a block of 32
bins can span the whole shadow of the image, rays can miss it on either side
or run along its edges, and bands are cut short.  The sweep takes sides from
2 to 37 (even and odd), 1 to 90 angles (axis-parallel only, 45 degrees, odd
counts, many full groups of 8) and detectors from one bin to wider than the image's diagonal, in
float32 (1e-5) and float64 (1e-12).  The error of each operator output is
measured against |W| |x| (|W|^T |y|), the scale of a sum's rounding: with a
few angles and one bin an output can be a near-cancelling sum of a handful of
random-sign terms, whose relative error is not a property of the kernel.
A block that loses its rays or rows gives an error of order one on this scale.

The packet diagonal is compared elementwise (same tolerances) at the deepest
level count the side allows (tiles up to the whole image), on detectors of
more than one bin: with a single bin some coefficients that a ray does see
lie near 1e-10 of the largest, below what float32 sums of squares resolve to
1e-5.  Packet basis functions that no ray sees (axis-parallel angle sets with
whole-image tiles) have coefficients that are zero in exact arithmetic; either side
computes them as exact zeros or as rounding noise (about 1e-32 of the largest
coefficient in float64, 1e-15 in float32).  Coefficients at most 1e-12 of the
largest are taken as that class on both sides: the other side must be there
too, far below any coefficient a ray sees.  The WMG apply (relative L2, same
tolerances) is compared where no coefficient falls in (0, 1e-12] of the
largest, since 1 / noise is noise on either side.
"""
import functools

import numpy as np
import pytest

from gpu_common import to_gpu, to_np
from oracle import joseph, wmg
from oracle.geometry import Geometry as OG
from oracle.projector import system_matrix

torch = pytest.importorskip("torch")
reco = pytest.importorskip("paper_1310_0956_amd")

pytestmark = pytest.mark.gpu

SIDES = (2, 3, 5, 8, 13, 14, 17, 24, 31, 37)
ANGLES = (1, 2, 3, 4, 6, 9, 45, 90)
TOL = {False: 1e-5, True: 1e-12}


def _bins(n):
    return sorted({1, n, int(n * 1.42) + 1, 2 * n + 5})


def _levels(n):
    """The most WMG levels n allows (2^(levels-1) divides n), at most 6."""
    lv = 1
    while lv < 6 and n % (1 << lv) == 0:
        lv += 1
    return lv


@functools.lru_cache(maxsize=4)
def _system(n, m, nb, jos):
    g = OG(n, m, nb)
    return (joseph.joseph_matrix(g) if jos else system_matrix(g)).tocsr()


def _scaled_err(got, want, scale):
    return np.linalg.norm(got - want) / np.linalg.norm(scale)


UNSEEN = 1e-12   # coefficients at most this fraction of the largest: unseen functions


def _check_diag(d, d_ref, tol):
    """Elementwise within tol above the unseen band; inside it on both sides below."""
    d = np.asarray(d, dtype=np.float64).ravel()
    d_ref = np.asarray(d_ref, dtype=np.float64).ravel()
    floor = UNSEEN * d_ref.max()
    low = d_ref <= floor
    assert np.all(np.abs(d[low]) <= floor), float(np.abs(d[low]).max())
    e = np.abs(d[~low] - d_ref[~low]) / d_ref[~low]
    assert e.max(initial=0.0) <= tol, float(e.max(initial=0.0))
    return bool(np.any((d_ref > 0) & low) or np.any((d > 0) & (d <= floor)))


@pytest.mark.parametrize("jos", [False, True], ids=["exact", "joseph"])
@pytest.mark.parametrize("n", SIDES)
def test_small_geometry_sweep(n, jos):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n))
    lv = _levels(n)
    proj = reco.PROJ_JOSEPH if jos else reco.PROJ_EXACT
    checked = 0
    for m in ANGLES:
        for nb in _bins(n):
            W = _system(n, m, nb, jos)
            Wa = abs(W)
            y = rng.standard_normal((m, nb))
            d_ref = wmg.packet_diagonal(W, n, lv - 1) if lv > 1 and nb > 1 else None
            for f64 in (False, True):
                dt = torch.float64 if f64 else torch.float32
                g = reco.Geometry(n, m, nb, lv, reco.F64 if f64 else reco.F32, projector=proj)
                xs, ys = to_gpu(x, dt), to_gpu(y, dt)
                x_dev, y_dev = to_np(xs).ravel(), to_np(ys).ravel()
                b = to_np(g.project(xs)).ravel()
                bt = to_np(g.backproject(ys)).ravel()
                eb = _scaled_err(b, W @ x_dev, Wa @ np.abs(x_dev))
                ebt = _scaled_err(bt, W.T @ y_dev, Wa.T @ np.abs(y_dev))
                if eb > TOL[f64] or ebt > TOL[f64]:
                    print(f"CASE n={n} m={m} nb={nb} f64={f64} joseph={jos}: forward {eb:.3e} "
                          f"backward {ebt:.3e}", flush=True)
                assert eb <= TOL[f64] and ebt <= TOL[f64]
                if d_ref is not None:
                    noisy = _check_diag(g.packet_diagonal(), d_ref, TOL[f64])
                    for lam in (0.0, 0.37) if not noisy else ():
                        z = to_np(g.wmg_apply(xs, lam=lam)).ravel()
                        z_ref = np.ravel(wmg.apply_additive_diag(x_dev, d_ref + lam, lv - 1))
                        assert np.linalg.norm(z - z_ref) <= TOL[f64] * np.linalg.norm(z_ref)
                checked += 1
    print(f"n={n} joseph={jos} levels={lv}: {checked} geometry/precision pairs", flush=True)
