"""GPU projectors with Joseph's kernel (RECO_PROJ_JOSEPH) against the Joseph oracle.

The kernels are the exact-length ones with other per-angle weight
coefficients; these tests compare W x, W^T y, the packet diagonal and the WMG
apply with the oracle's explicit Joseph matrix, check the adjoint identity of
the GPU pair, and run a float64 WMG-CGLS solve against the oracle's CG on the
same matrix.
"""
import functools

import numpy as np
import pytest

from gpu_common import check_diag_elementwise, print_case, rel, to_gpu, to_np
from oracle import joseph, solvers, wmg
from oracle.geometry import Geometry as OG

import inputs

torch = pytest.importorskip("torch")
reco = pytest.importorskip("paper_1310_0956_amd")

pytestmark = pytest.mark.gpu

# (n, m, nb, levels, f64): ragged sizes, the paper's 40x40 geometry, axis-only
# and 45-degree angle sets, a single angle and bin
CASES = [
    (24, 18, 35, 3, False),
    (40, 100, 40, 2, False),
    (64, 90, 64, 2, True),
    (48, 2, 70, 2, False),
    (32, 4, 45, 4, True),
    (16, 1, 1, 2, True),
    (14, 6, 33, 2, True),   # blocks whose first and last rays miss the image
    (160, 5, 227, 2, False),   # band windows wider than the LDS window: read from memory
    (128, 37, 182, 3, False),
    (64, 90, 91, 5, False),
    (128, 37, 182, 5, True),
    (64, 45, 91, 6, False),
    (64, 45, 91, 6, True),
]
TOL = {False: 1e-5, True: 1e-12}


@functools.lru_cache(maxsize=4)
def _J(n, m, nb):
    return joseph.joseph_matrix(OG(n, m, nb))


@functools.lru_cache(maxsize=4)
def _dJ(n, m, nb, L):
    return wmg.packet_diagonal(_J(n, m, nb), n, L)


def _img(n, seed):
    rng = np.random.default_rng(seed)
    return rng.random((n, n)) + (rng.random((n, n)) > 0.8)


@pytest.mark.parametrize("n,m,nb,lv,f64", CASES)
def test_joseph_operators_parity(n, m, nb, lv, f64):
    print_case("joseph operators", n, m, nb, lv, f64)
    dt = torch.float64 if f64 else torch.float32
    g = reco.Geometry(n, m, nb, lv, reco.F64 if f64 else reco.F32, projector=reco.PROJ_JOSEPH)
    J = _J(n, m, nb)
    xs = to_gpu(_img(n, 3), dt)
    x_dev = to_np(xs)
    b = to_np(g.project(xs))
    assert rel(b, J @ x_dev.ravel()) <= TOL[f64]
    ys = to_gpu(np.random.default_rng(4).standard_normal((m, nb)), dt)
    y_dev = to_np(ys)
    bt = to_np(g.backproject(ys))
    assert rel(bt, J.T @ y_dev.ravel()) <= TOL[f64]
    lhs = float(np.dot(b.ravel(), y_dev.ravel()))
    rhs = float(np.dot(x_dev.ravel(), bt.ravel()))
    assert abs(lhs - rhs) <= (1e-12 if f64 else 2e-6) * abs(lhs)
    L = lv - 1
    d_ref = _dJ(n, m, nb, L)
    check_diag_elementwise(g.packet_diagonal(), d_ref, TOL[f64])
    z = to_np(g.wmg_apply(xs, lam=0.0))
    assert rel(z, wmg.apply_additive_diag(x_dev, d_ref, L)) <= TOL[f64]


def test_joseph_differs_from_exact_lengths():
    """The projector choice reaches the kernels (a generic angle set differs)."""
    n, m, nb = 32, 30, 46
    print_case("joseph vs exact", n, m, nb)
    xs = to_gpu(_img(n, 5), torch.float64)
    bj = to_np(reco.Geometry(n, m, nb, 2, reco.F64, projector=reco.PROJ_JOSEPH).project(xs))
    be = to_np(reco.Geometry(n, m, nb, 2, reco.F64).project(xs))
    assert rel(bj, be) > 1e-3


def test_joseph_wmg_cgls_f64_matches_oracle():
    n, m, nb, lv = 64, 90, 64, 2
    print_case("joseph wmg-cgls f64", n, m, nb, lv)
    J = _J(n, m, nb)
    x_true = inputs.ellipse_phantom(n, 10, 0)
    b = J @ x_true.ravel()
    d = _dJ(n, m, nb, lv - 1)
    g = reco.Geometry(n, m, nb, lv, reco.F64, projector=reco.PROJ_JOSEPH)
    bg = to_gpu(b.reshape(m, nb), torch.float64)
    for precond in (reco.PRECOND_NONE, reco.PRECOND_WMG):
        M = (lambda v: wmg.apply_additive_diag(v, d, lv - 1)) if precond else None
        ref = solvers.pcgls(J, b, fixed_iters=10, precond=M)
        x, info = g.solve_cgls(bg, fixed_iters=10, precond=precond, history=True)
        assert info["iters"] == 10 and info["status"] == "ok"
        assert rel(to_np(x), ref.x) <= 1e-8, precond
        assert np.allclose(info["history"], ref.history, rtol=1e-8), precond
