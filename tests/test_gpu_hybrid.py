"""The hybrid wavelet multigrid cycle with exact coarsest solves on the GPU
against the oracle's HybridCycle (float64), alone and as the right
preconditioner of BiCGStab and GMRES.

Bars (float64): the cycle itself within 1e-9 of the oracle's (the coarsest
blocks are formed by different algorithms, Galerkin applies on the GPU and
sparse products in the oracle, and their factors amplify that rounding by
the blocks' condition numbers); BiCGStab iterates and residual histories
within 1e-8 over the first iterations (BiCGStab amplifies rounding ~30x per
iteration later, as for the diagonal preconditioner), GMRES within 1e-8.
"""
import numpy as np
import pytest

import inputs
from gpu_common import oracle_W, phantom_and_data, print_case, rel, to_gpu, to_np
from oracle import solvers, wmg

torch = pytest.importorskip("torch")
reco = pytest.importorskip("paper_1310_0956_amd")

pytestmark = pytest.mark.gpu

# (n, m, nb, levels, lam): the paper's 40^2 / 100 x 40 problem (one level),
# two and three levels, Tikhonov, and axis-only geometries whose coarsest
# blocks are singular (pivots dropped).  The factorisation runs in panels of
# 16 unknowns: blocks of 400, 64, 36 (a ragged last panel), 16 (one panel),
# 9 (less than one panel) and 36 with dropped pivots in every panel.
APPLY_CASES = [(40, 100, 40, 2, 0.0), (32, 24, 46, 3, 0.0), (32, 24, 46, 3, 0.2),
               (48, 30, 70, 4, 0.05), (16, 2, 9, 3, 0.0), (12, 6, 17, 3, 0.1),
               (24, 2, 35, 3, 0.0)]


@pytest.mark.parametrize("n,m,nb,lv,lam", APPLY_CASES)
def test_hybrid_apply_matches_oracle(n, m, nb, lv, lam):
    print_case("hybrid apply", n, m, nb, lv, lam)
    W = oracle_W(n, m, nb)
    cyc = wmg.HybridCycle(W, n, lv - 1, lam)
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    rng = np.random.default_rng(n + m)
    for k in range(2):
        r = W.T @ rng.standard_normal(m * nb) if k == 0 else rng.standard_normal(n * n)
        z = to_np(g.wmg_hybrid_apply(to_gpu(r.reshape(n, n), torch.float64), lam=lam))
        z_ref = cyc(r)
        print("hybrid apply rel err", rel(z, z_ref), "dropped",
              sum(int((~kp).sum()) for kp, _ in cyc.leaf.values()), flush=True)
        assert rel(z, z_ref) <= 1e-9


def test_hybrid_bicgstab_paper_problem_f64():
    """The paper's 40^2 / 100 x 40 problem and its 160^2 / 400 x 160 one
    (seeded ellipses, noiseless), WMG-BiCGStab with the hybrid cycle."""
    for n, m, nb, lv, E in [(40, 100, 40, 2, 6), (160, 400, 160, 3, 10)]:
        print_case("hybrid bicgstab", n, m, nb, lv)
        _, b = phantom_and_data(n, m, nb, E, 31 + n, dtype64=True)
        W = oracle_W(n, m, nb)
        cyc = wmg.HybridCycle(W, n, lv - 1)
        g = reco.Geometry(n, m, nb, lv, reco.F64)
        bg = to_gpu(b.reshape(m, nb), torch.float64)
        for k in (1, 3):
            ref = solvers.bicgstab_right(W, b, fixed_iters=k, precond=cyc)
            x, info = g.solve_bicgstab(bg, fixed_iters=k, precond=reco.PRECOND_WMG_HYBRID,
                                       history=True)
            dev = rel(to_np(x), ref.x)
            print(f"hybrid bicgstab {n}: {k} iterations dev {dev:.3e} relres {info['relres']:.4e}"
                  f" oracle {ref.relres:.4e}", flush=True)
            assert info["iters"] == k and info["status"] == "ok"
            assert dev <= 1e-8
            assert np.allclose(info["history"], ref.history, rtol=1e-8)


def test_hybrid_gmres_f64():
    n, m, nb, lv, lam = 32, 40, 46, 3, 0.0
    print_case("hybrid gmres", n, m, nb, lv)
    _, b = phantom_and_data(n, m, nb, 6, 41, noise=0.01, dtype64=True)
    W = oracle_W(n, m, nb)
    cyc = wmg.HybridCycle(W, n, lv - 1, lam)
    ref = solvers.gmres_right(W, b, fixed_iters=6, restart=4, precond=cyc)
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    x, info = g.solve_gmres(to_gpu(b.reshape(m, nb), torch.float64), fixed_iters=6, restart=4,
                            precond=reco.PRECOND_WMG_HYBRID)
    print("hybrid gmres dev", rel(to_np(x), ref.x), flush=True)
    assert rel(to_np(x), ref.x) <= 1e-8


def test_hybrid_f32_converges_like_oracle():
    """Float32 vectors (float64 factors): the same convergence as the oracle."""
    n, m, nb, lv = 64, 90, 64, 3
    print_case("hybrid f32", n, m, nb, lv)
    _, b = phantom_and_data(n, m, nb, 8, 51, noise=0.01)
    W = oracle_W(n, m, nb)
    cyc = wmg.HybridCycle(W, n, lv - 1)
    ref = solvers.bicgstab_right(W, b, fixed_iters=3, precond=cyc)
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    x, info = g.solve_bicgstab(to_gpu(b.reshape(m, nb), torch.float32), fixed_iters=3,
                               precond=reco.PRECOND_WMG_HYBRID)
    print("hybrid f32 dev", rel(to_np(x), ref.x), flush=True)
    assert rel(to_np(x), ref.x) <= 1e-4


def test_hybrid_rejected_where_unsupported():
    g = reco.Geometry(32, 20, 46, 3, reco.F32)
    b = torch.zeros((20, 46), dtype=torch.float32, device="cuda")
    with pytest.raises(reco.RecoError) as e:
        g.solve_cgls(b, precond=reco.PRECOND_WMG_HYBRID)
    assert e.value.status == reco.RECO_EINVAL
    g1 = reco.Geometry(32, 20, 46, 1, reco.F32)         # no wavelet level
    with pytest.raises(reco.RecoError) as e:
        g1.solve_bicgstab(b, precond=reco.PRECOND_WMG_HYBRID)
    assert e.value.status == reco.RECO_EINVAL
    g5 = reco.Geometry(32, 20, 46, 5, reco.F32)         # four levels: beyond the limit
    with pytest.raises(reco.RecoError) as e:
        g5.wmg_hybrid_apply(torch.zeros((32, 32), dtype=torch.float32, device="cuda"))
    assert e.value.status == reco.RECO_EINVAL
