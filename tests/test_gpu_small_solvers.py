"""GPU solvers on small geometries (float64, through the C ABI) against the
oracle's: a few iterations of CGLS, WMG-CGLS, WMG-GMRES and WMG-BiCGStab, with
and without Tikhonov regularisation, on images from 5 to 31 pixels whose
forward blocks span the image's whole shadow (rays that miss the image on
either side, axis-parallel-only and odd angle sets, unseen packet basis
functions).  Iterates within 1e-8 of the oracle's (relative L2).
"""
import numpy as np
import pytest

from gpu_common import oracle_W, oracle_d, print_case, rel, to_gpu, to_np
from oracle import solvers, wmg

torch = pytest.importorskip("torch")
reco = pytest.importorskip("paper_1310_0956_amd")

pytestmark = pytest.mark.gpu

# (n, m, nb, levels, lambda)
CASES = [(5, 3, 8, 1, 0.0), (13, 9, 19, 1, 0.0), (14, 6, 33, 2, 0.0), (24, 2, 35, 3, 0.0),
         (16, 4, 23, 3, 0.1), (31, 9, 45, 1, 0.0), (24, 9, 35, 2, 0.05)]


@pytest.mark.parametrize("n,m,nb,lv,lam", CASES)
def test_small_geometry_solvers_f64(n, m, nb, lv, lam):
    print_case("small solvers f64", n, m, nb, lv, lam)
    W = oracle_W(n, m, nb)
    b = np.random.default_rng(n * 100 + m).standard_normal(m * nb)
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    bg = to_gpu(b.reshape(m, nb), torch.float64)
    L = lv - 1
    d = oracle_d(n, m, nb, L)
    M = (lambda v: wmg.apply_additive_diag(v, d + lam, L)) if L > 0 else None
    pre = reco.PRECOND_WMG if L > 0 else reco.PRECOND_NONE
    runs = [
        ("cgls", solvers.pcgls(W, b, fixed_iters=6, lam=lam),
         g.solve_cgls(bg, fixed_iters=6, lam=lam, precond=reco.PRECOND_NONE)),
        ("wmg-cgls", solvers.pcgls(W, b, fixed_iters=6, lam=lam, precond=M),
         g.solve_cgls(bg, fixed_iters=6, lam=lam, precond=pre)),
        ("wmg-gmres", solvers.gmres_right(W, b, fixed_iters=6, restart=4, lam=lam, precond=M),
         g.solve_gmres(bg, fixed_iters=6, restart=4, lam=lam, precond=pre)),
        ("wmg-bicgstab", solvers.bicgstab_right(W, b, fixed_iters=3, lam=lam, precond=M),
         g.solve_bicgstab(bg, fixed_iters=3, lam=lam, precond=pre)),
    ]
    for name, ref, (x, info) in runs:
        dev = rel(to_np(x), ref.x)
        print(f"{name}: {info['iters']} iterations, status {info['status']}, dev {dev:.3e}", flush=True)
        assert info["status"] == "ok"
        assert dev <= 1e-8
