"""GPU BiCGStab (right preconditioned, on the normal equations) against the float64 oracle.

BiCGStab amplifies rounding far more than CGLS on these systems: on the
noiseless 64^2 case the oracle's own iterate after 10 iterations moves by
~2e-5 (relative) when its operator outputs carry relative errors of 1e-15,
growing ~30x per iteration from the 4th (CGLS: 1e-8 under 1e-13).  The
float64 tests therefore check the first iterations to 1e-8 (iterates and
residual histories) and later iterates within 10x the oracle's envelope under
relative 2^-53 operator perturbations (several seeds); tolerance-driven
solves are compared where that envelope is small (the same stopping
iteration).  At 512^2 (noisy data, 6 iterations to 1e-3) the envelope is 6e-14
and the float64 iterate is held to 1e-4 at the oracle's stopping iteration.
Float32 path: the first iterates within 1e-4, then convergence within three
iterations of the oracle's count to the same reconstruction error against the
true image (the oracle under float32-size perturbations: envelope 3e-4, same
iteration count and error).
"""
import numpy as np
import pytest

from gpu_common import oracle_W, oracle_d, phantom_and_data, print_case, rel, to_gpu, to_np
from oracle import solvers, wmg

torch = pytest.importorskip("torch")
reco = pytest.importorskip("paper_1310_0956_amd")

pytestmark = pytest.mark.gpu


def _minv(d, L):
    return lambda v: wmg.apply_additive_diag(v, d, L)


class _PerturbedW:
    """W whose products (W v and W^T r) pick up relative errors of up to eps."""

    def __init__(self, W, eps, seed):
        self.W, self.eps, self.g = W, eps, np.random.default_rng(seed)
        self.shape = W.shape

    def _noisy(self, y):
        return y * (1.0 + self.eps * self.g.uniform(-1.0, 1.0, y.shape))

    def __matmul__(self, v):
        return self._noisy(self.W @ v)

    @property
    def T(self):
        outer = self

        class _T:
            def __matmul__(self, r):
                return outer._noisy(outer.W.T @ r)
        return _T()


def _envelope(W, b, ref_x, seeds=3, **kw):
    return max(rel(solvers.bicgstab_right(_PerturbedW(W, 2.0 ** -53, s), b, **kw).x, ref_x)
               for s in range(seeds))


def test_bicgstab_tiny64_f64_matches_oracle():
    """64^2, 90 angles x 64 bins, 10 ellipses, noiseless, float64: plain and WMG."""
    n, m, nb, lv = 64, 90, 64, 2
    print_case("tiny64 f64 bicgstab")
    _, b = phantom_and_data(n, m, nb, 10, 0, dtype64=True)
    W = oracle_W(n, m, nb)
    d = oracle_d(n, m, nb, lv - 1)
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    bg = to_gpu(b.reshape(m, nb), torch.float64)
    for precond in (reco.PRECOND_NONE, reco.PRECOND_WMG):
        M = _minv(d, lv - 1) if precond else None
        ref4 = solvers.bicgstab_right(W, b, fixed_iters=4, precond=M)
        x, info = g.solve_bicgstab(bg, fixed_iters=4, precond=precond, history=True)
        assert info["iters"] == 4 and info["matvecs"] == 8 and info["status"] == "ok"
        assert rel(to_np(x), ref4.x) <= 1e-8, precond
        assert np.allclose(info["history"], ref4.history, rtol=1e-8), precond
        ref = solvers.bicgstab_right(W, b, fixed_iters=10, precond=M)
        x, info = g.solve_bicgstab(bg, fixed_iters=10, precond=precond, history=True)
        env = _envelope(W, b, ref.x, fixed_iters=10, precond=M)
        dev = rel(to_np(x), ref.x)
        print("tiny64 bicgstab precond", precond, "dev", dev, "oracle float64 envelope", env,
              flush=True)
        assert info["iters"] == 10 and dev <= max(10 * env, 1e-8), precond
    # the preconditioner helps
    r_plain = solvers.bicgstab_right(W, b, fixed_iters=10).relres
    r_wmg = solvers.bicgstab_right(W, b, fixed_iters=10, precond=_minv(d, lv - 1)).relres
    assert r_wmg < r_plain


def test_bicgstab_tikhonov_and_tolerance_f64():
    n, m, nb, lv = 32, 40, 46, 3
    print_case("bicgstab tikhonov f64")
    _, b = phantom_and_data(n, m, nb, 6, 5, noise=0.01, dtype64=True)
    W = oracle_W(n, m, nb)
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    bg = to_gpu(b.reshape(m, nb), torch.float64)
    # lambda = 0.2: well conditioned, 10 iterations to 1e-6 (oracle envelope 4e-9)
    lam = 0.2
    M = _minv(oracle_d(n, m, nb, lv - 1) + lam, lv - 1)
    ref = solvers.bicgstab_right(W, b, tol=1e-6, max_iter=200, lam=lam, precond=M)
    x, info = g.solve_bicgstab(bg, tol=1e-6, max_iter=200, lam=lam, history=True)
    assert ref.converged and info["status"] == "ok"
    assert info["iters"] == ref.iters and info["matvecs"] == ref.matvecs
    assert rel(to_np(x), ref.x) <= 1e-7
    assert np.allclose(info["history"], ref.history, rtol=1e-7)
    # lambda = 0: ~140 iterations to 1e-6 with an envelope of 1e-3; the first five
    lam = 0.0
    M = _minv(oracle_d(n, m, nb, lv - 1), lv - 1)
    ref = solvers.bicgstab_right(W, b, fixed_iters=5, lam=lam, precond=M)
    x, info = g.solve_bicgstab(bg, fixed_iters=5, lam=lam, history=True)
    assert rel(to_np(x), ref.x) <= 1e-8
    assert np.allclose(info["history"], ref.history, rtol=1e-8)


CT = (512, 360, 725, 3)


@pytest.fixture(scope="module")
def ct512():
    n, m, nb, lv = CT
    x_true, b = phantom_and_data(n, m, nb, 20, 1000, noise=0.01)
    return x_true, b


def test_bicgstab_ct512_f64_to_tolerance(ct512):
    """Full 512^2 workload through the float64 instantiation."""
    n, m, nb, lv = CT
    print_case("ct512 f64 wmg-bicgstab")
    _, b = ct512
    W = oracle_W(n, m, nb)
    ref = solvers.bicgstab_right(W, b, tol=1e-3, precond=_minv(oracle_d(n, m, nb, lv - 1), lv - 1))
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    x, info = g.solve_bicgstab(to_gpu(b.reshape(m, nb), torch.float64), tol=1e-3, history=True)
    assert ref.converged and info["status"] == "ok" and info["iters"] == ref.iters
    assert rel(to_np(x), ref.x) <= 1e-4
    assert np.allclose(info["history"][:4], ref.history[:4], rtol=1e-8)


def test_bicgstab_ct512_f32(ct512):
    n, m, nb, lv = CT
    print_case("ct512 f32 wmg-bicgstab")
    x_true, b = ct512
    W = oracle_W(n, m, nb)
    M = _minv(oracle_d(n, m, nb, lv - 1), lv - 1)
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    bg = to_gpu(b.reshape(m, nb), torch.float32)
    ref2 = solvers.bicgstab_right(W, b, fixed_iters=2, precond=M)
    x2, _ = g.solve_bicgstab(bg, fixed_iters=2)
    assert rel(to_np(x2), ref2.x) <= 1e-4
    ref = solvers.bicgstab_right(W, b, tol=1e-3, precond=M)
    x, info = g.solve_bicgstab(bg, tol=1e-3)
    print("ct512 f32 bicgstab iters", info["iters"], "oracle", ref.iters, flush=True)
    assert info["status"] == "ok" and abs(info["iters"] - ref.iters) <= 3
    e_gpu, e_ref = rel(to_np(x), x_true.ravel()), rel(ref.x, x_true.ravel())
    assert e_gpu <= 1.05 * e_ref + 1e-3, (e_gpu, e_ref)
    # deterministic: the same solve twice gives the same bits
    x_again, info2 = g.solve_bicgstab(bg, tol=1e-3)
    assert info2["iters"] == info["iters"] and torch.equal(x, x_again)


def test_bicgstab_edge_cases():
    n, m, nb, lv = 32, 24, 46, 2
    print_case("bicgstab edge cases")
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    zero = torch.zeros((m, nb), dtype=torch.float32, device="cuda")
    x, info = g.solve_bicgstab(zero, tol=1e-3)
    assert info["iters"] == 0 and info["status"] == "ok"
    assert float(torch.abs(x).max()) == 0.0
    bad = zero.clone()
    bad[3, 7] = float("nan")
    x, info = g.solve_bicgstab(bad, tol=1e-3)
    assert info["status"] == "enumeric"
    # iteration cap: not converged, x is the iterate at the cap
    _, b = phantom_and_data(n, m, nb, 5, 3, noise=0.01)
    W = oracle_W(n, m, nb)
    d = oracle_d(n, m, nb, lv - 1)
    x, info = g.solve_bicgstab(to_gpu(b.reshape(m, nb), torch.float32), tol=1e-12, max_iter=5)
    assert info["status"] == "not_converged" and info["iters"] == 5
    ref = solvers.bicgstab_right(W, b, fixed_iters=5, precond=_minv(d, lv - 1))
    assert rel(to_np(x), ref.x) <= 1e-4
    with pytest.raises(reco.RecoError):
        g.solve_bicgstab(to_gpu(b.reshape(m, nb), torch.float32), tol=-1.0)
