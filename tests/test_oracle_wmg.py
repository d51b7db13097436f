"""Pins of the oracle WMG preconditioners.

  * the packet diagonal equals diag(H_L W^T W H_L^T) from dense matrices (+ lam),
    and has the mirror, reflection and quarter-turn symmetries of the geometry;
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
from oracle.projector import angle_block, system_matrix


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


def _quadrant_to_tile_local(dq, L):
    """Packet diagonal from the quadrant layout (packet (pr, pc) in block
    [pr cs, (pr + 1) cs) x [pc cs, (pc + 1) cs), cs = n / 2^L) to the tile-local
    layout: tile (tx, ty) of 2^L x 2^L pixels holds its own coefficients, the
    packet's row and column bits read least significant level first."""
    n = dq.shape[0]
    T = 1 << L
    out = np.empty_like(dq)
    for iy in range(n):
        for ix in range(n):
            ly, lx = iy & (T - 1), ix & (T - 1)
            row, col = iy >> L, ix >> L
            for lev in range(1, L + 1):
                row += ((ly >> (lev - 1)) & 1) * (n >> lev)
                col += ((lx >> (lev - 1)) & 1) * (n >> lev)
            out[iy, ix] = dq[row, col]
    return out


@pytest.mark.parametrize("n,m,nb,L", [(16, 8, 23, 2), (12, 8, 17, 2), (12, 7, 17, 2),
                                      (24, 12, 35, 3), (6, 4, 9, 0), (16, 6, 16, 1),
                                      (16, 2, 23, 2), (16, 1, 23, 2), (20, 9, 29, 2)])
def test_packet_diagonal_symmetries(n, m, nb, L):
    """The geometry's symmetries, on which the device computation of d rests.
    With bins centred on the rotation centre a tile and its mirror through the
    image centre have equal sums at every angle; angle m - k is angle k
    reflected left-right (on tile (tx, ty): angle k's sums of X T =
    (N - 1 - tx, ty)); with m even, angle m/2 - k is angle k reflected about
    the diagonal (the transposed tile (ty, tx), packet row and column
    exchanged) and angle k + m/2 is angle k turned by a quarter (tile
    R T = (ty, N - 1 - tx), row and column exchanged).  So with A the sum over
    angles 0 .. floor(m/4) (m even) or 0 .. (m - 1)/2 (m odd), angle 0 and, when
    4 divides m, angle m/4 weighted 1/2, over the tiles t < ceil(N^2 / 2):
    d(T) = A(T) + A(X T) (+ A(T^T)^T + A(R T)^T for m even)."""
    g = Geometry(n, m, nb)
    full = _quadrant_to_tile_local(wmg.packet_diagonal_by_angles(g, L), L)
    if m % 2 == 0:
        wts = {k: 1.0 for k in range(m // 4 + 1)}
        if m % 4 == 0:
            wts[m // 4] = 0.5
    else:
        wts = {k: 1.0 for k in range((m - 1) // 2 + 1)}
    wts[0] = 0.5
    A = sum(w * _quadrant_to_tile_local(wmg.packet_diagonal([angle_block(g, k)], n, L), L)
            for k, w in wts.items())
    T, N = 1 << L, n >> L
    nt = N * N
    nh = (nt + 1) // 2

    def tile(t):   # the computed tile standing for tile t, its sums
        t = t if t < nh else nt - 1 - t
        ty, tx = divmod(t, N)
        return A[ty * T:(ty + 1) * T, tx * T:(tx + 1) * T]

    got = np.empty_like(full)
    for ty in range(N):
        for tx in range(N):
            blk = tile(ty * N + tx) + tile(ty * N + (N - 1 - tx))
            if m % 2 == 0:
                blk = blk + tile(tx * N + ty).T + tile((N - 1 - tx) * N + ty).T
            got[ty * T:(ty + 1) * T, tx * T:(tx + 1) * T] = blk
    assert np.allclose(got, full, rtol=1e-12, atol=1e-14 * full.max())
    # fewer angles than m are summed once m > 2
    assert len(wts) < m or m <= 2


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


# --- hybrid and additive cycles (Section 3.1.2, eq. wmg and the hybrid variant) ---

def _projection(A, R):
    """P = R^T (R A R^T)^-1 R: the A-orthogonal projection onto range(R^T), times A^-1."""
    return R.T @ np.linalg.solve(R @ A @ R.T, R)


def _real_system(n, m, nb, lam):
    Wd = system_matrix(Geometry(n, m, nb)).toarray()
    return Wd.T @ Wd + lam * np.eye(n * n)


def _cycle_matrix(cyc, N):
    return np.column_stack([cyc(e) for e in np.eye(N)])


class _HybridWithoutUpdate(wmg.WaveletCycle):
    """Planted mistake: the hybrid cycle with its residual update r2 = r - A e dropped."""

    def _cycle(self, node, r):
        if node[0] == "leaf":
            return wmg.coarsest_solve(node[1][0], r)
        _, A, kids = node
        R, sub = kids["LL"]
        e = R.T @ self._cycle(sub, R @ r)
        for name in self.ORDER[1:]:
            R, sub = kids[name]
            e = e + R.T @ self._cycle(sub, R @ r)   # r, not r - A e
        return e


class _HybridHighFirst(wmg.WaveletCycle):
    """Planted mistake: the three wavelet corrections before the LL one."""

    def _cycle(self, node, r):
        if node[0] == "leaf":
            return wmg.coarsest_solve(node[1][0], r)
        _, A, kids = node
        e = np.zeros_like(r)
        for name in self.ORDER[1:]:
            R, sub = kids[name]
            e = e + R.T @ self._cycle(sub, R @ r)
        r2 = r - A @ e
        R, sub = kids["LL"]
        return e + R.T @ self._cycle(sub, R @ r2)


def _hybrid_error_propagation(A, n):
    """One level: E = (I - sum_{LH,HL,HH} P_id A)(I - P_LL A)."""
    ops = haar.step_operators_2d(n)
    I = np.eye(n * n)
    P = {k: _projection(A, ops[k].toarray()) for k in ("LL", "LH", "HL", "HH")}
    high = P["LH"] + P["HL"] + P["HH"]
    return (I - high @ A) @ (I - P["LL"] @ A)


def _additive_error_propagation(A, n):
    ops = haar.step_operators_2d(n)
    S = sum(_projection(A, ops[k].toarray()) for k in ("LL", "LH", "HL", "HH"))
    return np.eye(n * n) - S @ A


@pytest.mark.parametrize("n,m,nb,lam", [(8, 16, 12, 0.1), (8, 7, 11, 0.0), (16, 24, 23, 0.02)])
def test_hybrid_error_propagation(n, m, nb, lam):
    """Hybrid WTG on a real geometry: I - M^-1 A equals the product of the LL
    projection and the summed wavelet projections, LL first."""
    A = _real_system(n, m, nb, lam)
    want = _hybrid_error_propagation(A, n)
    scale = np.abs(want).max()
    got = np.eye(n * n) - _cycle_matrix(wmg.WaveletCycle(A, n, 1, "hybrid"), n * n) @ A
    assert np.abs(got - want).max() <= 1e-9 * scale
    # planted mistakes in the oracle: both must fail this pin
    for bad in (_HybridWithoutUpdate, _HybridHighFirst):
        wrong = np.eye(n * n) - _cycle_matrix(bad(A, n, 1, "hybrid"), n * n) @ A
        assert np.abs(wrong - want).max() > 1e-3 * scale, bad.__name__


@pytest.mark.parametrize("n,m,nb,lam", [(8, 16, 12, 0.1), (16, 24, 23, 0.0)])
def test_additive_error_propagation(n, m, nb, lam):
    """Additive WTG: I - M^-1 A = I - sum over the four subbands of P_id A."""
    A = _real_system(n, m, nb, lam)
    want = _additive_error_propagation(A, n)
    scale = np.abs(want).max()
    got = np.eye(n * n) - _cycle_matrix(wmg.WaveletCycle(A, n, 1, "additive"), n * n) @ A
    assert np.abs(got - want).max() <= 1e-9 * scale
    # the hybrid cycle (one extra residual update) is a different operator
    hyb = np.eye(n * n) - _cycle_matrix(wmg.WaveletCycle(A, n, 1, "hybrid"), n * n) @ A
    assert np.abs(hyb - want).max() > 1e-3 * scale


@pytest.mark.parametrize("n,L", [(8, 2), (16, 2), (16, 3)])
def test_recursive_additive_cycle_is_packet_block_jacobi(n, L):
    """The additive cycle recursed to depth L with exact coarsest solves equals the
    block-Jacobi preconditioner of the packet basis, sum_p V_p (V_p^T K V_p)^-1 V_p^T,
    built independently from the packet matrix H_L and the sparse W."""
    W = system_matrix(Geometry(n, 3 * n // 2, n + 3))
    K = (W.T @ W).toarray() + 0.05 * np.eye(n * n)
    cyc = wmg.WaveletCycle(K, n, L, "additive")
    F = sla.cholesky(K, lower=False)
    blocks = wmg.galerkin_blocks(F, n, L)
    rng = np.random.default_rng(12)
    for _ in range(3):
        r = rng.standard_normal(n * n)
        a = cyc(r)
        b = wmg.apply_additive_exact(r, blocks, n, L)
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)


def test_recursive_hybrid_two_levels():
    """Two levels: the hybrid cycle's error propagation factors as the top-level
    product with each subband's exact projection replaced by that subband's own
    (one level down) hybrid cycle, I - (Q_H + Q_LL - Q_H A Q_LL) A, where
    Q_id = R_id^T B_id R_id and I - B_id A_id is the one-level formula on A_id."""
    n, lam = 8, 0.05
    A = _real_system(n, 12, 12, lam)
    ops = haar.step_operators_2d(n)
    Q = {}
    for k in ("LL", "LH", "HL", "HH"):
        R = ops[k].toarray()
        Ak = R @ A @ R.T
        Ek = _hybrid_error_propagation(Ak, n // 2)
        Bk = np.linalg.solve(Ak.T, (np.eye(Ak.shape[0]) - Ek).T).T   # (I - E_k) A_k^-1
        Q[k] = R.T @ Bk @ R
    QH = Q["LH"] + Q["HL"] + Q["HH"]
    Minv = Q["LL"] + QH - QH @ A @ Q["LL"]
    got = _cycle_matrix(wmg.WaveletCycle(A, n, 2, "hybrid"), n * n)
    assert np.abs(got - Minv).max() <= 1e-9 * np.abs(Minv).max()
    bad = _cycle_matrix(_HybridWithoutUpdate(A, n, 2, "hybrid"), n * n)
    assert np.abs(bad - Minv).max() > 1e-3 * np.abs(Minv).max()


# --- the matrix-free hybrid cycle and unseen coarsest unknowns ---

@pytest.mark.parametrize("n,m,nb,L,lam", [(8, 10, 12, 1, 0.0), (16, 12, 23, 2, 0.0),
                                          (16, 20, 23, 2, 0.3), (16, 9, 16, 3, 0.05)])
def test_matrix_free_hybrid_equals_dense_cycle(n, m, nb, L, lam):
    """HybridCycle (Galerkin operators applied through W and the step
    operators, coarsest blocks from W R_P^T) equals WaveletCycle(mode="hybrid")
    built from the dense K."""
    W = system_matrix(Geometry(n, m, nb))
    K = (W.T @ W).toarray() + lam * np.eye(n * n)
    dense = wmg.WaveletCycle(K, n, L, "hybrid")
    mf = wmg.HybridCycle(W, n, L, lam)
    rng = np.random.default_rng(21)
    for _ in range(3):
        r = rng.standard_normal(n * n)
        a, b = dense(r), mf(r)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)
    # the Galerkin apply of a node is R_P K R_P^T
    R = wmg.subband_restriction(n, ("HL",) * min(L, 1))
    u = rng.standard_normal(R.shape[0])
    want = R @ (K @ (R.T @ u))
    assert np.allclose(mf.galerkin_apply(("HL",) * min(L, 1), u), want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_subband_restriction_orthonormal_and_matches_packet_transform():
    """R_P has orthonormal rows, and R_P x is packet P of the L-level packet
    transform (quadrant layout) of x."""
    n, L = 16, 2
    x = np.random.default_rng(3).standard_normal((n, n))
    c = haar.packet_transform(x, L)
    cs = n >> L
    names = ("LL", "LH", "HL", "HH")
    q = {"LL": (0, 0), "LH": (0, 1), "HL": (1, 0), "HH": (1, 1)}
    for a in names:
        for b in names:
            R = wmg.subband_restriction(n, (a, b))
            assert np.allclose((R @ R.T).toarray(), np.eye(cs * cs), atol=1e-14)
            row = q[a][0] * (n >> 1) + q[b][0] * (n >> 2)
            col = q[a][1] * (n >> 1) + q[b][1] * (n >> 2)
            assert np.allclose((R @ x.ravel()).reshape(cs, cs), c[row:row + cs, col:col + cs],
                               atol=1e-13)


def test_coarsest_solve_drops_unseen_unknowns():
    """A positive semi-definite block (two unseen unknowns, one more that
    repeats a combination of others): the dropped unknowns get a zero correction,
    the result solves A e = r for r in the range of A, and with nothing to drop
    it is the plain Cholesky solve."""
    rng = np.random.default_rng(5)
    G = rng.standard_normal((30, 12))
    G[:, [2, 7]] = 0.0                          # two unseen unknowns
    G[:, 9] = G[:, 0] - 0.5 * G[:, 4]           # a dependent one (dropped at its pivot)
    A = G.T @ G
    keep, Lk = wmg.coarsest_factor(A)
    assert list(np.nonzero(~keep)[0]) == [2, 7, 9]
    r = A @ rng.standard_normal(12)              # in the range of A
    e = wmg.coarsest_solve((keep, Lk), r)
    assert e[2] == 0.0 and e[7] == 0.0 and e[9] == 0.0
    assert np.allclose(A @ e, r, atol=1e-10 * np.abs(r).max())
    B = A + np.eye(12)
    fac = wmg.coarsest_factor(B)
    assert fac[0].all()
    assert np.allclose(wmg.coarsest_solve(fac, r), np.linalg.solve(B, r), rtol=1e-12, atol=1e-12)


def test_coarsest_factor_elimination_matches_lapack():
    """The explicit elimination (used when a pivot is dropped) equals LAPACK's
    Cholesky on a positive definite block; a planted wrong pivot order fails."""
    rng = np.random.default_rng(6)
    G = rng.standard_normal((40, 10))
    A = G.T @ G
    A[3, 3] *= 1.0 + 1e-9
    Lref = np.linalg.cholesky(A)
    # force the elimination path: one unseen unknown appended
    A2 = np.zeros((11, 11))
    A2[:10, :10] = A
    keep, Lk = wmg.coarsest_factor(A2)
    assert keep[:10].all() and not keep[10]
    assert np.allclose(Lk, Lref, rtol=1e-12, atol=1e-12)
    assert not np.allclose(Lk, np.linalg.cholesky(A[::-1, ::-1]), atol=1e-6)


def test_hybrid_cycle_with_unseen_pixels():
    """Two axis directions with a detector narrower than the image leave its
    corners unseen (with many angles every pixel is seen at the angle
    perpendicular to its position): the coarsest blocks are singular, the cycle
    still runs, dropped unknowns get no correction, and the dense and
    matrix-free cycles agree."""
    n, m, nb, L = 16, 2, 9, 2
    W = system_matrix(Geometry(n, m, nb))
    assert (np.asarray(abs(W).sum(axis=0)).ravel() == 0).any()   # unseen pixels exist
    mf = wmg.HybridCycle(W, n, L)
    assert sum(int((~k).sum()) for k, _ in mf.leaf.values()) > 0
    K = (W.T @ W).toarray()
    dense = wmg.WaveletCycle(K, n, L, "hybrid")
    r = W.T @ np.random.default_rng(9).standard_normal(m * nb)
    a, b = dense(r), mf(r)
    assert np.all(np.isfinite(b))
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(a)
