"""Pins of the oracle WMG preconditioners.

  * the packet diagonal equals diag(H_L W^T W H_L^T) from dense matrices (+ lam);
  * additive-exact inverts K when K = H_L^T B H_L with B block diagonal over packets;
  * additive-diagonal inverts K when B is diagonal;
  * the hybrid cycle also inverts such K exactly (the packet subspaces are then
    K-orthogonal, so every correction is the exact one);
  * on a real geometry each preconditioner lowers the condition number.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import haar, wmg
from oracle.geometry import Geometry
from oracle.projector import system_matrix


@pytest.mark.parametrize("n,m,nb,L,lam", [(8, 10, 12, 1, 0.0), (16, 12, 23, 2, 0.0),
                                          (16, 9, 16, 3, 0.25), (8, 6, 11, 2, 1.0)])
def test_packet_diagonal_brute_force(n, m, nb, L, lam):
    g = Geometry(n, m, nb)
    W = system_matrix(g)
    d = wmg.packet_diagonal(W, n, L, lam)
    H = haar.packet_matrix(n, L).toarray()
    Wd = W.toarray()
    want = np.diag(H @ (Wd.T @ Wd + lam * np.eye(n * n)) @ H.T)
    assert np.allclose(d.ravel(), want, rtol=1e-13, atol=1e-15)
    d2 = wmg.packet_diagonal_by_angles(g, L, lam)
    assert np.allclose(d2, d, rtol=1e-13, atol=1e-15)


def _block_diag_K(n, L, seed, diagonal=False):
    rng = np.random.default_rng(seed)
    H = haar.packet_matrix(n, L).toarray()
    B = np.zeros((n * n, n * n))
    for cols in wmg.packet_columns(n, L):
        k = len(cols)
        if diagonal:
            blk = np.diag(rng.uniform(0.5, 3.0, k))
        else:
            G = rng.standard_normal((k, k))
            blk = G @ G.T + k * np.eye(k)
        B[np.ix_(cols, cols)] = blk
    return H.T @ B @ H, B


@pytest.mark.parametrize("n,L", [(8, 1), (8, 2), (16, 2)])
def test_additive_exact_inverts_block_diagonal(n, L):
    K, _ = _block_diag_K(n, L, 3)
    # galerkin blocks from K via a factor K = F^T F
    F = sla.cholesky(K, lower=False)
    blocks = wmg.galerkin_blocks(F, n, L)
    r = np.random.default_rng(4).standard_normal(n * n)
    z = wmg.apply_additive_exact(r, blocks, n, L)
    assert np.allclose(K @ z, r, atol=1e-10)


@pytest.mark.parametrize("n,L", [(8, 1), (16, 3)])
def test_additive_diag_inverts_diagonal(n, L):
    K, B = _block_diag_K(n, L, 5, diagonal=True)
    H = haar.packet_matrix(n, L).toarray()
    d = np.diag(H @ K @ H.T).reshape(n, n)
    r = np.random.default_rng(6).standard_normal(n * n)
    z = wmg.apply_additive_diag(r, d, L)
    assert np.allclose(K @ z, r, atol=1e-11)


@pytest.mark.parametrize("n,L", [(8, 1), (8, 2)])
@pytest.mark.parametrize("mode", ["multiplicative", "hybrid", "additive"])
def test_cycles_invert_block_diagonal(n, L, mode):
    K, _ = _block_diag_K(n, L, 7)
    cyc = wmg.WaveletCycle(K, n, L, mode)
    r = np.random.default_rng(8).standard_normal(n * n)
    assert np.allclose(K @ cyc(r), r, atol=1e-10)


def test_multiplicative_error_propagation_is_product_of_projections():
    """eq. wmg: one WTG sweep propagates the error by prod_id (I - P_id A)."""
    n = 8
    g = Geometry(n, 16, 12)
    Wd = system_matrix(g).toarray()
    A = Wd.T @ Wd + 0.1 * np.eye(n * n)
    cyc = wmg.WaveletCycle(A, n, 1, "multiplicative")
    ops = haar.step_operators_2d(n)
    E = np.eye(n * n)
    for name in ("LL", "LH", "HL", "HH"):
        R = ops[name].toarray()
        P = R.T @ np.linalg.solve(R @ A @ R.T, R)
        E = (np.eye(n * n) - P @ A) @ E
    Minv = np.column_stack([cyc(e) for e in np.eye(n * n)])
    assert np.allclose(np.eye(n * n) - Minv @ A, E, atol=1e-9)


def _cond_sym(A):
    ev = np.linalg.eigvals(A)
    return np.abs(ev).max() / np.abs(ev).min()


def test_preconditioners_reduce_condition_number():
    n, L = 16, 2
    g = Geometry(n, 40, 23)
    W = system_matrix(g)
    Wd = W.toarray()
    K = Wd.T @ Wd
    d = wmg.packet_diagonal(W, n, L)
    Mdiag = np.column_stack([wmg.apply_additive_diag(e, d, L) for e in np.eye(n * n)])
    blocks = wmg.galerkin_blocks(W, n, L)
    Mex = np.column_stack([wmg.apply_additive_exact(e, blocks, n, L) for e in np.eye(n * n)])
    k0 = _cond_sym(K)
    assert _cond_sym(K @ Mdiag) < k0 / 3
    assert _cond_sym(K @ Mex) < k0 / 3
    # the additive-diagonal operator is symmetric positive definite
    assert np.allclose(Mdiag, Mdiag.T, atol=1e-12)
    assert np.linalg.eigvalsh(0.5 * (Mdiag + Mdiag.T)).min() > 0
