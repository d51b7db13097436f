"""GPU parity of the projectors over a sweep of small geometries (through the C
ABI, against the CPU float64 oracle's W).

Small images stress the forward projector's per-block set-up: a block of 32
bins can span the whole shadow of the image, rays can miss it on either side
or run along its edges, and bands are cut short.  The sweep takes sides from
2 to 37 (even and odd), 1 to 9 angles (axis-parallel only, 45 degrees, odd
counts) and detectors from one bin to wider than the image's diagonal, in
float32 (1e-5) and float64 (1e-12).  The error of each operator output is
measured against |W| |x| (|W|^T |y|), the scale of a sum's rounding: with a
few angles and one bin an output can be a near-cancelling sum of a handful of
random-sign terms, whose relative error is not a property of the kernel.
A block that loses its rays or rows gives an error of order one on this scale.
The packet diagonal is compared elementwise, and the WMG apply in relative L2
(same tolerances), where one wavelet level fits and the detector has more than
one bin: with a single bin
some coefficients are zero in exact arithmetic and come out as rounding noise
(about 1e-32 of the largest in the float64 oracle, 1e-15 in float32), where
neither side's value means anything.
"""
import numpy as np
import pytest

from gpu_common import check_diag_elementwise, oracle_d, to_gpu, to_np
from oracle import wmg
from oracle.geometry import Geometry as OG
from oracle.projector import system_matrix

torch = pytest.importorskip("torch")
reco = pytest.importorskip("paper_1310_0956_amd")

pytestmark = pytest.mark.gpu

SIDES = (2, 3, 5, 8, 13, 14, 17, 24, 31, 37)
ANGLES = (1, 2, 3, 4, 6, 9)
TOL = {False: 1e-5, True: 1e-12}


def _bins(n):
    return sorted({1, n, int(n * 1.42) + 1, 2 * n + 5})


@pytest.mark.parametrize("n", SIDES)
def test_small_geometry_sweep(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n))
    checked = 0
    for m in ANGLES:
        for nb in _bins(n):
            W = system_matrix(OG(n, m, nb))
            y = rng.standard_normal((m, nb))
            for f64 in (False, True):
                dt = torch.float64 if f64 else torch.float32
                lv = 2 if n % 2 == 0 else 1
                g = reco.Geometry(n, m, nb, lv, reco.F64 if f64 else reco.F32)
                xs, ys = to_gpu(x, dt), to_gpu(y, dt)
                x_dev, y_dev = to_np(xs), to_np(ys)
                b = to_np(g.project(xs)).ravel()
                bt = to_np(g.backproject(ys)).ravel()
                Wa = abs(W)
                eb = np.linalg.norm(b - W @ x_dev.ravel()) / np.linalg.norm(Wa @ np.abs(x_dev.ravel()))
                ebt = (np.linalg.norm(bt - W.T @ y_dev.ravel())
                       / np.linalg.norm(Wa.T @ np.abs(y_dev.ravel())))
                if eb > TOL[f64] or ebt > TOL[f64]:
                    print(f"CASE n={n} m={m} nb={nb} f64={f64}: forward {eb:.3e} "
                          f"backward {ebt:.3e}", flush=True)
                assert eb <= TOL[f64] and ebt <= TOL[f64]
                if lv == 2 and nb > 1:
                    d_ref = oracle_d(n, m, nb, 1)
                    check_diag_elementwise(g.packet_diagonal(), d_ref, TOL[f64])
                    for lam in (0.0, 0.37):
                        z = to_np(g.wmg_apply(xs, lam=lam)).ravel()
                        z_ref = np.ravel(wmg.apply_additive_diag(x_dev, d_ref + lam, 1))
                        assert np.linalg.norm(z - z_ref) <= TOL[f64] * np.linalg.norm(z_ref)
                checked += 1
    print(f"n={n}: {checked} geometry/precision pairs", flush=True)
