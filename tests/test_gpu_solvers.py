"""GPU solver parity against the float64 oracle at the same iteration count.

Float64 path: iterates within 1e-4 of the oracle's at the oracle's stopping
iteration for tolerance-driven solves, within 1e-8 over the first 10
iterations, and for the 50-iteration noiseless runs within 10x the oracle's own
float64-rounding envelope (the oracle perturbed by relative 2^-53 errors in the
vectors it keeps, several seeds; that envelope itself reaches 1e-4 there).

Float32 path (float32 projectors and vectors, float64 scalars and reductions):
CG on these noisy normal equations amplifies perturbations of its vectors by
~10x per iteration from about the 6th iteration on.  The float64 oracle run
with every kept vector rounded to float32 (and nothing else changed) already
moves by 3.2e-2 at the 14th WMG-CGLS iteration of the 512^2 case, so no
float32-storage implementation can hold 1e-4 there; that figure is met by the
float64 instantiation only.  The float32 bar is an envelope measured on the
oracle: at the test's geometry the GPU projector's and backprojector's
relative error against the oracle's W and W^T is measured first (eps); the
oracle is then rerun with every kept vector given a relative Gaussian error of
size eps and rounded to float32, over five seeds, at the GPU's iteration
count K, and the GPU iterate must lie within 3x the largest deviation seen.
The tests also check (a) early iterates to 1e-5, (c) the same reconstruction
error against the true image within 10%, and (d) stopping within 2 iterations
of the oracle, and print K, the deviation, eps and the envelope.
"""
import math

import numpy as np
import pytest

from gpu_common import (f32_envelope, oracle_W, oracle_d, operator_eps, phantom_and_data, print_case,
                        rel, to_gpu, to_np)
from oracle import solvers, wmg

torch = pytest.importorskip("torch")
reco = pytest.importorskip("paper_1310_0956_amd")

pytestmark = pytest.mark.gpu


def _minv(d, L):
    return lambda v: wmg.apply_additive_diag(v, d, L)


def _f32(v):
    return v.astype(np.float32).astype(np.float64)


def _perturb(eps, seed):
    """Storage model: every kept vector picks up a relative error of up to eps."""
    g = np.random.default_rng(seed)
    return lambda v: v * (1.0 + eps * g.uniform(-1.0, 1.0, np.shape(v)))


def _envelope(run, ref_x, eps, seeds=3):
    """Largest deviation of the oracle from itself under rounding-size perturbations."""
    return max(rel(run(_perturb(eps, s)).x, ref_x) for s in range(seeds))


F32_EPS, F64_EPS = 2.0 ** -24, 2.0 ** -53


def test_tiny64_f64_fifty_iterations():
    """64^2, 90 angles x 64 bins, 10 ellipses, noiseless, float64: SIRT, CGLS, WMG-CGLS x 50."""
    n, m, nb, lv = 64, 90, 64, 2
    print_case("tiny64 f64 solvers")
    x_true, b = phantom_and_data(n, m, nb, 10, 0, dtype64=True)
    W = oracle_W(n, m, nb)
    d = oracle_d(n, m, nb, lv - 1)
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    bg = to_gpu(b.reshape(m, nb), torch.float64)
    ref = solvers.sirt(W, b, fixed_iters=50)
    x, info = g.solve_sirt(bg, fixed_iters=50, history=True)
    assert info["iters"] == 50 and info["status"] == "ok"
    assert rel(to_np(x), ref.x) <= 1e-8
    assert np.allclose(info["history"], ref.history, rtol=1e-8)
    for precond in (reco.PRECOND_NONE, reco.PRECOND_WMG):
        M = _minv(d, lv - 1) if precond else None
        ref10 = solvers.pcgls(W, b, fixed_iters=10, precond=M)
        x, info = g.solve_cgls(bg, fixed_iters=10, precond=precond)
        assert rel(to_np(x), ref10.x) <= 1e-8, precond
        ref = solvers.pcgls(W, b, fixed_iters=50, precond=M)
        x, info = g.solve_cgls(bg, fixed_iters=50, precond=precond, history=True)
        assert info["iters"] == 50
        env = _envelope(lambda h: solvers.pcgls(W, b, fixed_iters=50, precond=M, store=h), ref.x,
                        F64_EPS, seeds=4)
        dev = rel(to_np(x), ref.x)
        print("tiny64 cgls precond", precond, "dev", dev, "oracle float64 envelope", env, flush=True)
        assert dev <= max(10 * env, 1e-4), precond
        # residual histories agree while the iteration is well conditioned
        assert np.allclose(info["history"][:10], ref.history[:10], rtol=1e-8)
    # the preconditioner helps: lower residual after the same 50 iterations
    r_plain = solvers.pcgls(W, b, fixed_iters=50).relres
    r_wmg = solvers.pcgls(W, b, fixed_iters=50, precond=_minv(d, lv - 1)).relres
    assert r_wmg < r_plain


CT = (512, 360, 725, 3)


@pytest.fixture(scope="module")
def ct512():
    n, m, nb, lv = CT
    x_true, b = phantom_and_data(n, m, nb, 20, 1000, noise=0.01)
    return x_true, b


@pytest.mark.parametrize("precond", [1, 0])
def test_ct512_f64_cgls_to_tolerance(ct512, precond):
    """Full 512^2 workload through the float64 instantiation: spec parity."""
    n, m, nb, lv = CT
    print_case("ct512 f64 cgls", precond)
    x_true, b = ct512
    W = oracle_W(n, m, nb)
    M = _minv(oracle_d(n, m, nb, lv - 1), lv - 1) if precond else None
    ref = solvers.pcgls(W, b, tol=1e-3, precond=M)
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    x, info = g.solve_cgls(to_gpu(b.reshape(m, nb), torch.float64), tol=1e-3, precond=precond,
                           history=True)
    assert info["status"] == "ok" and info["iters"] == ref.iters
    assert rel(to_np(x), ref.x) <= 1e-4
    assert np.allclose(info["history"][:8], ref.history[:8], rtol=1e-8)


def test_ct512_f64_wmg_gmres_to_tolerance(ct512):
    n, m, nb, lv = CT
    print_case("ct512 f64 wmg-gmres30")
    x_true, b = ct512
    W = oracle_W(n, m, nb)
    ref = solvers.gmres_right(W, b, tol=1e-3, restart=30, precond=_minv(oracle_d(n, m, nb, lv - 1), lv - 1))
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    x, info = g.solve_gmres(to_gpu(b.reshape(m, nb), torch.float64), tol=1e-3, restart=30)
    assert info["status"] == "ok" and info["iters"] == ref.iters
    assert rel(to_np(x), ref.x) <= 1e-4


@pytest.mark.parametrize("precond", [1, 0])
def test_ct512_f32_cgls(ct512, precond):
    n, m, nb, lv = CT
    print_case("ct512 f32 cgls", precond)
    x_true, b = ct512
    W = oracle_W(n, m, nb)
    M = _minv(oracle_d(n, m, nb, lv - 1), lv - 1) if precond else None
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    bg = to_gpu(b.reshape(m, nb), torch.float32)
    e_fwd, e_bwd = operator_eps(g, W, x_true, b.reshape(m, nb))
    eps = max(e_fwd, e_bwd)
    # (a) early iterates
    x5, _ = g.solve_cgls(bg, fixed_iters=5, precond=precond)
    assert rel(to_np(x5), solvers.pcgls(W, b, fixed_iters=5, precond=M).x) <= 1e-5
    # (d) stopping iteration
    ref = solvers.pcgls(W, b, tol=1e-3, precond=M)
    x, info = g.solve_cgls(bg, tol=1e-3, precond=precond)
    K = info["iters"]
    assert info["status"] == "ok" and abs(K - ref.iters) <= 2
    # (b) iterate at K within 3x the oracle's float32 envelope at the measured operator error
    refK = solvers.pcgls(W, b, fixed_iters=K, precond=M)
    spread = f32_envelope(lambda h: solvers.pcgls(W, b, fixed_iters=K, precond=M, store=h),
                           refK.x, eps)
    dev = rel(to_np(x), refK.x)
    print(f"ct512 f32 cgls precond={precond}: K {K} (oracle {ref.iters}) dev {dev:.3e} "
          f"operator eps fwd {e_fwd:.3e} bwd {e_bwd:.3e} envelope {spread:.3e}", flush=True)
    assert dev <= 3 * spread
    # (c) reconstruction quality
    e_gpu, e_ref = rel(to_np(x), x_true), rel(refK.x, x_true)
    assert abs(e_gpu - e_ref) <= 0.1 * e_ref


def test_ct512_f32_wmg_gmres(ct512):
    n, m, nb, lv = CT
    print_case("ct512 f32 wmg-gmres30")
    x_true, b = ct512
    W = oracle_W(n, m, nb)
    M = _minv(oracle_d(n, m, nb, lv - 1), lv - 1)
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    e_fwd, e_bwd = operator_eps(g, W, x_true, b.reshape(m, nb))
    eps = max(e_fwd, e_bwd)
    x, info = g.solve_gmres(to_gpu(b.reshape(m, nb), torch.float32), tol=1e-3, restart=30)
    K = info["iters"]
    ref = solvers.gmres_right(W, b, tol=1e-3, restart=30, precond=M)
    assert info["status"] == "ok" and abs(K - ref.iters) <= 2
    refK = solvers.gmres_right(W, b, fixed_iters=K, restart=30, precond=M)
    spread = f32_envelope(lambda h: solvers.gmres_right(W, b, fixed_iters=K, restart=30,
                                                         precond=M, store=h), refK.x, eps)
    dev = rel(to_np(x), refK.x)
    print(f"ct512 f32 wmg-gmres30: K {K} (oracle {ref.iters}) dev {dev:.3e} operator eps "
          f"fwd {e_fwd:.3e} bwd {e_bwd:.3e} envelope {spread:.3e}", flush=True)
    assert dev <= 3 * spread


def test_ct512_sirt_fixed(ct512):
    n, m, nb, lv = CT
    print_case("ct512 sirt x30")
    x_true, b = ct512
    W = oracle_W(n, m, nb)
    ref = solvers.sirt(W, b, fixed_iters=30)
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    x, info = g.solve_sirt(to_gpu(b.reshape(m, nb), torch.float32), fixed_iters=30)
    assert rel(to_np(x), ref.x) <= 1e-4


@pytest.mark.parametrize("restart", [3, 7])
def test_gmres_restarts_and_tikhonov_f64(restart):
    n, m, nb, lv = 32, 40, 46, 3
    print_case("gmres restarts", restart)
    _, b = phantom_and_data(n, m, nb, 6, 5, noise=0.01, dtype64=True)
    W = oracle_W(n, m, nb)
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    for lam in (0.0, 0.2):
        d = oracle_d(n, m, nb, lv - 1) + lam
        ref = solvers.gmres_right(W, b, tol=1e-4, restart=restart, lam=lam, max_iter=60,
                                  precond=_minv(d, lv - 1))
        x, info = g.solve_gmres(to_gpu(b.reshape(m, nb), torch.float64), tol=1e-4,
                                restart=restart, lam=lam, max_iter=60)
        assert info["iters"] == ref.iters
        assert info["matvecs"] == ref.matvecs
        assert rel(to_np(x), ref.x) <= 1e-8


def test_cgls_tikhonov_matches_oracle():
    n, m, nb, lv = 48, 60, 68, 3
    print_case("cgls tikhonov")
    lam = 0.3
    W = oracle_W(n, m, nb)
    d = oracle_d(n, m, nb, lv - 1) + lam
    for f64 in (True, False):
        _, b = phantom_and_data(n, m, nb, 7, 9, noise=0.02, dtype64=f64)
        g = reco.Geometry(n, m, nb, lv, reco.F64 if f64 else reco.F32)
        ref = solvers.pcgls(W, b, fixed_iters=25, lam=lam, precond=_minv(d, lv - 1))
        x, info = g.solve_cgls(to_gpu(b.reshape(m, nb), torch.float64 if f64 else torch.float32),
                               fixed_iters=25, lam=lam)
        assert rel(to_np(x), ref.x) <= (1e-8 if f64 else 1e-4)


def test_edge_cases():
    n, m, nb, lv = 32, 24, 46, 2
    print_case("solver edge cases")
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    zero = torch.zeros((m, nb), dtype=torch.float32, device="cuda")
    for fn in (g.solve_cgls, g.solve_gmres, g.solve_sirt):
        x, info = fn(zero, tol=1e-3)
        assert info["iters"] == 0 and info["status"] == "ok"
        assert float(torch.abs(x).max()) == 0.0
    bad = zero.clone()
    bad[3, 7] = float("nan")
    for fn in (g.solve_cgls, g.solve_gmres, g.solve_sirt):
        x, info = fn(bad, tol=1e-3)
        assert info["status"] == "enumeric"
    # iteration cap: not converged, x is the iterate at the cap
    _, b = phantom_and_data(n, m, nb, 5, 3, noise=0.01)
    W = oracle_W(n, m, nb)
    d = oracle_d(n, m, nb, lv - 1)
    x, info = g.solve_cgls(to_gpu(b.reshape(m, nb), torch.float32), tol=1e-12, max_iter=7)
    assert info["status"] == "not_converged" and info["iters"] == 7
    ref = solvers.pcgls(W, b, fixed_iters=7, precond=_minv(d, lv - 1))
    assert rel(to_np(x), ref.x) <= 1e-4
    with pytest.raises(reco.RecoError):
        g.solve_cgls(to_gpu(b.reshape(m, nb), torch.float32), tol=-1.0)
    with pytest.raises(reco.RecoError):
        g.solve_gmres(to_gpu(b.reshape(m, nb), torch.float32), restart=0)
