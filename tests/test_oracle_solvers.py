"""Pins of the oracle solvers on tiny systems.

  * PCGLS iterate k minimises ||b - W x||^2 + lam ||x||^2 over the preconditioned
    Krylov space span{(M^-1 K)^i M^-1 W^T b, i < k} (brute force: explicit basis and a
    dense least-squares solve); the converged iterate equals numpy lstsq;
  * GMRES iterate k minimises ||f - K M^-1 u|| over u in span{(K M^-1)^i f, i < k};
    with restart >= N it returns K^-1 f;
  * SIRT iterate k equals sum_{i<k} S^i C W^T R b with S = I - C W^T R W;
  * BiCGStab: each step makes s Petrov-Galerkin orthogonal to the shadow vector
    (<rhat, s> = 0) and r = s - omega t orthogonal to t (omega minimises ||s - omega t||);
    the recursive residual equals f - K x; the iterates converge to the dense solve;
    with the exact preconditioner M^-1 = K^-1 one step solves the system.
"""
import numpy as np
import pytest

from oracle import solvers, wmg
from oracle.geometry import Geometry
from oracle.projector import system_matrix


def _tiny(n=8, m=20, nb=12, seed=0):
    g = Geometry(n, m, nb)
    W = system_matrix(g)
    x = np.random.default_rng(seed).random(g.N)
    b = W @ x + 0.01 * np.random.default_rng(seed + 1).standard_normal(g.M)
    return g, W, b


def _krylov_basis(op, v0, k):
    V = [v0]
    for _ in range(k - 1):
        V.append(op(V[-1]))
    Q, _ = np.linalg.qr(np.column_stack(V))
    return Q


@pytest.mark.parametrize("lam,use_prec", [(0.0, False), (0.0, True), (0.3, True)])
def test_pcgls_minimises_over_krylov_space(lam, use_prec):
    g, W, b = _tiny()
    Wd = W.toarray()
    K = Wd.T @ Wd + lam * np.eye(g.N)
    if use_prec:
        d = wmg.packet_diagonal(W, g.n, 2, lam)
        Minv = lambda v: wmg.apply_additive_diag(v, d, 2)  # noqa: E731
    else:
        Minv = lambda v: v  # noqa: E731
    f = Wd.T @ b
    for k in range(1, 7):
        res = solvers.pcgls(W, b, lam=lam, precond=Minv, fixed_iters=k)
        Q = _krylov_basis(lambda v: Minv(K @ v), Minv(f), k)
        A = np.vstack([Wd @ Q, np.sqrt(lam) * Q]) if lam else Wd @ Q
        rhs = np.concatenate([b, np.zeros(g.N)]) if lam else b
        y = np.linalg.lstsq(A, rhs, rcond=None)[0]
        want = Q @ y
        assert np.linalg.norm(res.x - want) <= 1e-9 * np.linalg.norm(want)


def test_pcgls_converges_to_least_squares():
    g, W, b = _tiny(n=6, m=24, nb=10)
    want = np.linalg.lstsq(W.toarray(), b, rcond=None)[0]
    res = solvers.pcgls(W, b, tol=1e-12, max_iter=500)
    assert res.converged
    assert np.linalg.norm(res.x - want) <= 1e-8 * np.linalg.norm(want)
    d = wmg.packet_diagonal(W, g.n, 1)
    res2 = solvers.pcgls(W, b, tol=1e-12, max_iter=500,
                         precond=lambda v: wmg.apply_additive_diag(v, d, 1))
    assert np.linalg.norm(res2.x - want) <= 1e-8 * np.linalg.norm(want)
    assert res2.iters < res.iters


@pytest.mark.parametrize("use_prec", [False, True])
def test_gmres_minimises_over_krylov_space(use_prec):
    g, W, b = _tiny()
    Wd = W.toarray()
    K = Wd.T @ Wd
    if use_prec:
        d = wmg.packet_diagonal(W, g.n, 1)
        Minv = lambda v: wmg.apply_additive_diag(v, d, 1)  # noqa: E731
    else:
        Minv = lambda v: v  # noqa: E731
    f = Wd.T @ b
    for k in range(1, 7):
        res = solvers.gmres_right(W, b, restart=30, precond=Minv, fixed_iters=k)
        Q = _krylov_basis(lambda v: K @ Minv(v), f, k)
        KM = np.column_stack([K @ Minv(Q[:, i]) for i in range(k)])
        y = np.linalg.lstsq(KM, f, rcond=None)[0]
        want = Minv(Q @ y)
        assert np.linalg.norm(res.x - want) <= 1e-8 * np.linalg.norm(want)
        assert abs(res.relres - np.linalg.norm(f - K @ res.x) / np.linalg.norm(f)) < 1e-10


def test_gmres_full_restart_is_exact_and_restarts_progress():
    g, W, b = _tiny(n=4, m=12, nb=6)
    Wd = W.toarray()
    K = Wd.T @ Wd
    f = Wd.T @ b
    res = solvers.gmres_right(W, b, restart=g.N, fixed_iters=g.N)
    assert np.linalg.norm(K @ res.x - f) <= 1e-8 * np.linalg.norm(f)
    short = solvers.gmres_right(W, b, restart=3, tol=1e-6, max_iter=400)
    assert short.converged
    assert np.linalg.norm(K @ short.x - f) <= 2e-6 * np.linalg.norm(f)


def test_sirt_closed_form():
    g, W, b = _tiny()
    Wd = W.toarray()
    R, C = solvers.sirt_weights(W)
    S = np.eye(g.N) - (C[:, None] * Wd.T) @ (R[:, None] * Wd)
    v = C * (Wd.T @ (R * b))
    acc = np.zeros(g.N)
    P = np.eye(g.N)
    for k in range(1, 8):
        acc = acc + P @ v
        P = S @ P
        res = solvers.sirt(W, b, fixed_iters=k)
        assert np.allclose(res.x, acc, rtol=1e-12, atol=1e-13)
    # relres_k is the size of the k-th correction relative to the first
    res = solvers.sirt(W, b, fixed_iters=5)
    x4 = solvers.sirt(W, b, fixed_iters=4).x
    assert abs(res.history[-1] - np.linalg.norm(res.x - x4) / np.linalg.norm(v)) < 1e-12


def test_sirt_zero_rows_get_zero_weight():
    g = Geometry(8, 6, 16)   # outer bins miss the image
    W = system_matrix(g)
    R, C = solvers.sirt_weights(W)
    rs = np.asarray(W.sum(axis=1)).ravel()
    assert (rs == 0).any()
    assert (R[rs == 0] == 0).all() and (R[rs > 0] > 0).all()


def _prec(g, W, use_prec, L=1):
    if not use_prec:
        return None
    d = wmg.packet_diagonal(W, g.n, L)
    return lambda v: wmg.apply_additive_diag(v, d, L)  # noqa: E731


@pytest.mark.parametrize("lam,use_prec", [(0.0, False), (0.0, True), (0.3, True)])
def test_bicgstab_step_properties_and_true_residual(lam, use_prec):
    g, W, b = _tiny()
    Wd = W.toarray()
    K = Wd.T @ Wd + lam * np.eye(g.N)
    f = Wd.T @ b
    seen = []

    def cb(i, v):
        sc = np.linalg.norm(v["rhat"]) * np.linalg.norm(v["s"])
        assert abs(v["rhat"] @ v["s"]) <= 1e-9 * sc
        if v["omega"] != 0.0:
            assert abs(v["r"] @ v["t"]) <= 1e-9 * np.linalg.norm(v["r"]) * np.linalg.norm(v["t"])
            # omega minimises ||s - w t||: nearby values do no better
            for dw in (1e-3, -1e-3):
                assert np.linalg.norm(v["s"] - (v["omega"] + dw) * v["t"]) >= np.linalg.norm(v["r"])
        true_r = f - K @ v["x"]
        assert np.linalg.norm(v["r"] - true_r) <= 1e-9 * np.linalg.norm(f)
        seen.append(i)

    res = solvers.bicgstab_right(W, b, lam=lam, precond=_prec(g, W, use_prec), fixed_iters=8,
                                 callback=cb)
    assert seen == list(range(1, res.iters + 1)) and res.iters >= 6
    for k, rr in enumerate(res.history):
        assert rr >= 0.0


@pytest.mark.parametrize("lam,use_prec", [(0.0, False), (0.0, True), (0.3, True)])
def test_bicgstab_converges_to_dense_solve(lam, use_prec):
    g, W, b = _tiny()
    Wd = W.toarray()
    K = Wd.T @ Wd + lam * np.eye(g.N)
    want = np.linalg.solve(K, Wd.T @ b)
    res = solvers.bicgstab_right(W, b, tol=1e-12, max_iter=2000, lam=lam,
                                 precond=_prec(g, W, use_prec))
    assert res.converged and res.matvecs == 2 * res.iters
    assert np.linalg.norm(res.x - want) <= 1e-7 * np.linalg.norm(want)


def test_bicgstab_exact_preconditioner_solves_in_one_step():
    g, W, b = _tiny(n=4, m=12, nb=6)
    Wd = W.toarray()
    K = Wd.T @ Wd + 0.1 * np.eye(g.N)
    Kinv = np.linalg.inv(K)
    res = solvers.bicgstab_right(W, b, tol=1e-10, max_iter=5, lam=0.1, precond=lambda v: Kinv @ v)
    assert res.converged and res.iters == 1
    assert np.linalg.norm(res.x - Kinv @ (Wd.T @ b)) <= 1e-10 * np.linalg.norm(res.x)
