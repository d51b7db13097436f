"""WMG preconditioners on the normal equations (oracle).

System operator K = W^T W + lam I (eq. sys_ne, eq. sys_reg with the squared
Tikhonov reading).  Let V_p denote the columns of H_L^T that belong to packet p
(one coarsest-grid subproblem of Section 3.1.3; 4^L of them, each with
(n/2^L)^2 unknowns).  The Galerkin coarse operator of a subproblem
(eq. galerkin and the WTG box of Section 3.1.2) is A_p = V_p^T K V_p.

Variants:
  * additive_exact: M^-1 = sum_p V_p A_p^-1 V_p^T.  This is the additive form of
    the wavelet two-grid scheme that Section 3.1.2 names, recursed to the
    coarsest level, with exact coarsest solves (Cholesky, as in Section 4.1).
  * additive_diag:  M^-1 = H_L^T diag(1/d) H_L with d_q = e_q^T H_L K H_L^T e_q
    = ||W H_L^T e_q||^2 + lam, i.e. A_p replaced by its diagonal.  1/d := 0
    where d = 0.  This is the reading used by the GPU path (the coarsest
    problems are too large for dense factorisation at the benchmark sizes).
  * WaveletCycle: the paper's multiplicative WTG (eq. wmg) and its hybrid
    variant (LL correction, one residual update, then LH, HL, HH from that
    residual; Section 3.1.2), recursed with exact coarsest solves.

Parity status: packet_diagonal pinned by brute force against dense
diag(H_L W^T W H_L^T) on small grids; the additive variants pinned by the
block-diagonal exactness property (K = H_L^T B H_L with B block diagonal is
inverted exactly).  WaveletCycle: on real projection matrices the one-level
error propagation I - M^-1 A is pinned against its closed form for every mode
(multiplicative: the product of the four A-orthogonal projections of eq. wmg;
hybrid: (I - sum_{LH,HL,HH} P_id A)(I - P_LL A); additive: I - sum_id P_id A,
with P_id = R_id^T (R_id A R_id^T)^-1 R_id); the two-level hybrid cycle against
the same formula with each subband's projection replaced by its own one-level
cycle; the additive cycle recursed to depth L against the packet-basis
block-Jacobi operator built from H_L (apply_additive_exact).  Planted mistakes
(the hybrid residual update dropped, the wavelet corrections taken before the
LL one) fail these pins.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import haar
from .geometry import Geometry
from .projector import angle_block


def packet_diagonal(W_blocks, n: int, L: int, lam: float = 0.0) -> np.ndarray:
    """d in quadrant layout [n][n]: squared column norms of W H_L^T, plus lam.

    W_blocks: a CSR matrix W or an iterable of row blocks of W (e.g. per angle).
    """
    HT = haar.packet_matrix(n, L).T.tocsr()
    if sp.issparse(W_blocks):
        W_blocks = [W_blocks]
    d = np.zeros(n * n)
    for Wk in W_blocks:
        Y = (Wk @ HT).tocsr()
        d += np.asarray(Y.multiply(Y).sum(axis=0)).ravel()
    return (d + lam).reshape(n, n)


def packet_diagonal_by_angles(g: Geometry, L: int, lam: float = 0.0) -> np.ndarray:
    """packet_diagonal streaming one angle block at a time (bounded memory)."""
    return packet_diagonal((angle_block(g, k) for k in range(g.m)), g.n, L, lam)


def apply_additive_diag(r: np.ndarray, d: np.ndarray, L: int) -> np.ndarray:
    """z = H_L^T diag(1/d) H_L r (1/d := 0 where d == 0)."""
    n = d.shape[0]
    c = haar.packet_transform(np.asarray(r, dtype=np.float64).reshape(n, n), L)
    inv = np.zeros_like(d)
    nz = d != 0.0
    inv[nz] = 1.0 / d[nz]
    return haar.packet_adjoint(c * inv, L).ravel()


def packet_columns(n: int, L: int) -> list[np.ndarray]:
    """For each packet p, the quadrant-layout flat indices of its coefficients."""
    cs = n >> L
    idx = np.arange(n * n).reshape(n, n)
    out = []
    for pr in range(1 << L):
        for pc in range(1 << L):
            out.append(idx[pr * cs:(pr + 1) * cs, pc * cs:(pc + 1) * cs].ravel())
    return out


def galerkin_blocks(W: sp.csr_matrix, n: int, L: int, lam: float = 0.0):
    """Cholesky factors of A_p = (W V_p)^T (W V_p) + lam I for every packet p.

    W may be the sparse projection matrix or any dense factor F with K = F^T F.
    """
    HT = haar.packet_matrix(n, L).T.tocsc()
    out = []
    for cols in packet_columns(n, L):
        WV = W @ HT[:, cols]
        WV = WV.toarray() if sp.issparse(WV) else np.asarray(WV)
        A = WV.T @ WV + lam * np.eye(len(cols))
        out.append((cols, sla.cho_factor(A, lower=True)))
    return out


def apply_additive_exact(r: np.ndarray, blocks, n: int, L: int) -> np.ndarray:
    """z = sum_p V_p A_p^-1 V_p^T r."""
    c = haar.packet_transform(np.asarray(r, dtype=np.float64).reshape(n, n), L).ravel()
    out = np.zeros_like(c)
    for cols, fac in blocks:
        out[cols] = sla.cho_solve(fac, c[cols])
    return haar.packet_adjoint(out.reshape(n, n), L).ravel()


class WaveletCycle:
    """One wavelet multigrid cycle with exact coarsest solves (Section 3.1.2-3.1.3).

    A cycle approximately solves K e = r with zero initial guess.  At a level
    with operator A, the four Galerkin operators A_id = R_id A R_id^T use the
    step operators R_id of eq. 1of4 - 4of4, and each coarse problem is treated
    by the same cycle one level down (exact Cholesky solve at the coarsest level).

    mode="multiplicative" (the WTG box, error propagation eq. wmg):
        for id in LL, LH, HL, HH: e += R_id^T cycle(A_id, R_id (r - A e))
    mode="hybrid" (the variant the experiments use, Section 3.1.2):
        e = R_LL^T cycle(A_LL, R_LL r); r' = r - A e;
        e += sum over LH, HL, HH of R_id^T cycle(A_id, R_id r')
    mode="additive":
        e = sum over all four of R_id^T cycle(A_id, R_id r)
    Operators are formed densely, so this is for small grids only.
    """

    ORDER = ("LL", "LH", "HL", "HH")

    def __init__(self, K: np.ndarray, n: int, L: int, mode: str = "hybrid"):
        assert mode in ("multiplicative", "hybrid", "additive")
        self.n, self.L, self.mode = n, L, mode
        self._leaves = []
        self.tree = self._build(np.asarray(K, dtype=np.float64), n, L)
        scale = max(float(np.diag(A).max()) for A, _ in self._leaves)
        for A, slot in self._leaves:
            slot.append(coarsest_factor(A, scale))

    def _build(self, A, s, levels):
        if levels == 0:
            slot = []                  # filled with the factor once all leaves are known
            self._leaves.append((A, slot))
            return ("leaf", slot)
        ops = haar.step_operators_2d(s)
        kids = {}
        for name in self.ORDER:
            R = ops[name].toarray()
            kids[name] = (R, self._build(R @ A @ R.T, s // 2, levels - 1))
        return ("node", A, kids)

    def _cycle(self, node, r):
        if node[0] == "leaf":
            return coarsest_solve(node[1][0], r)
        _, A, kids = node
        e = np.zeros_like(r)
        if self.mode == "multiplicative":
            for name in self.ORDER:
                R, sub = kids[name]
                e = e + R.T @ self._cycle(sub, R @ (r - A @ e))
        elif self.mode == "hybrid":
            R, sub = kids["LL"]
            e = R.T @ self._cycle(sub, R @ r)
            r2 = r - A @ e
            for name in self.ORDER[1:]:
                R, sub = kids[name]
                e = e + R.T @ self._cycle(sub, R @ r2)
        else:
            for name in self.ORDER:
                R, sub = kids[name]
                e = e + R.T @ self._cycle(sub, R @ r)
        return e

    def __call__(self, r):
        return self._cycle(self.tree, np.asarray(r, dtype=np.float64).ravel())


# ---------------------------------------------------------------------------
# Exact coarsest solves with unseen directions
# ---------------------------------------------------------------------------
# A coarsest Galerkin block A = (W V)^T (W V) + lam I is only positive
# semi-definite when lam = 0: a basis function that no ray sees has a zero
# row and column, and with few rays the seen ones can be linearly dependent.
# Reading (the paper's Cholesky solve, Section 4.1, on a singular block; the
# 1/0 := 0 rule of the diagonal case extended): the block is factored by
# Cholesky in its natural order, and an unknown whose pivot (the diagonal of
# the remaining Schur complement) is at most DROP_REL times the block's
# largest diagonal entry is dropped: its column is not eliminated and its
# correction is zero.  For a positive semi-definite block such a column of
# the Schur complement is zero up to rounding, so for r in the range of A the
# result still solves A e = r.  With no pivot dropped this is the plain
# Cholesky solve.  The threshold is relative to the largest diagonal entry of
# all coarsest blocks of the hierarchy (`scale`): the rounding that forming a
# block leaves in it is relative to the operator K, not to that block.
DROP_REL = 1e-12


def coarsest_factor(A: np.ndarray, scale: float | None = None):
    """(kept mask, lower Cholesky factor of the kept unknowns) of a Galerkin block;
    pivots at most DROP_REL * scale (default: the block's largest diagonal) are dropped."""
    A = np.array(A, dtype=np.float64)
    c = A.shape[0]
    if scale is None:
        scale = float(np.diag(A).max()) if c else 0.0
    thr = DROP_REL * max(scale, 0.0)
    try:   # fast path: LAPACK, accepted when it drops nothing
        Lf = sla.cholesky(A, lower=True)
        if c == 0 or float((np.diag(Lf) ** 2).min()) > thr:
            return np.ones(c, dtype=bool), Lf
    except np.linalg.LinAlgError:
        pass
    S = A.copy()                       # Schur complement, updated in place
    Lm = np.zeros_like(A)
    keep = np.zeros(c, dtype=bool)
    for k in range(c):
        piv = S[k, k]
        if piv <= thr:
            continue                   # dropped: not eliminated
        keep[k] = True
        col = S[k:, k] / np.sqrt(piv)
        Lm[k:, k] = col
        S[k + 1:, k + 1:] -= np.outer(col[1:], col[1:])
    return keep, Lm[np.ix_(keep, keep)]


def coarsest_solve(factor, r: np.ndarray) -> np.ndarray:
    """e = A^-1 r on the kept unknowns (two triangular solves), 0 on the dropped."""
    keep, Lk = factor
    r = np.asarray(r, dtype=np.float64)
    e = np.zeros_like(r)
    if keep.any():
        y = sla.solve_triangular(Lk, r[keep], lower=True)
        e[keep] = sla.solve_triangular(Lk.T, y, lower=False)
    return e


def subband_restriction(n: int, path) -> sp.csr_matrix:
    """R_P for a path of subband names, coarsest-level last: the product of the
    step operators of eq. 1of4 - 4of4 at the successive grid sizes (an
    (n / 2^l)^2 x n^2 matrix with orthonormal rows)."""
    R = sp.identity(n * n, format="csr")
    s = n
    for name in path:
        R = (haar.step_operators_2d(s)[name] @ R).tocsr()
        s //= 2
    return R


class HybridCycle:
    """The hybrid wavelet multigrid cycle of WaveletCycle(mode="hybrid"),
    matrix free: the Galerkin operator of a node P of the recursion,
    A_P = R_P K R_P^T with K = W^T W + lam I (eq. galerkin), is applied as
    R_P (W^T (W (R_P^T u))) + lam u, and only the coarsest operators are formed
    (densely, from the sparse W R_P^T) and factored (Cholesky, Section 4.1;
    unseen directions as in coarsest_factor, relative to the largest diagonal
    entry of all coarsest blocks).

    cycle(P, r):  P at depth L: e = A_P^-1 r
                  else: e = R_LL^T cycle(P LL, R_LL r);  r' = r - A_P e;
                        e += sum over LH, HL, HH of R_id^T cycle(P id, R_id r')
    with R_id the step operators at the node's grid size (Section 3.1.2, the
    hybrid variant; recursion of Section 3.1.3)."""

    ORDER = ("LL", "LH", "HL", "HH")

    def __init__(self, W: sp.csr_matrix, n: int, L: int, lam: float = 0.0):
        self.W, self.WT = W.tocsr(), W.T.tocsr()
        self.n, self.L, self.lam = n, L, float(lam)
        self.R = {}
        blocks = {}
        self._paths((), 0, blocks)
        scale = max(float(np.diag(A).max()) for A in blocks.values())
        self.leaf = {p: coarsest_factor(A, scale) for p, A in blocks.items()}

    def _paths(self, path, depth, blocks):
        self.R[path] = subband_restriction(self.n, path)
        if depth == self.L:
            G = (self.W @ self.R[path].T).tocsc()
            blocks[path] = (G.T @ G).toarray() + self.lam * np.eye(G.shape[1])
            return
        for name in self.ORDER:
            self._paths(path + (name,), depth + 1, blocks)

    def galerkin_apply(self, path, u):
        """A_P u = R_P (W^T (W (R_P^T u))) + lam u."""
        R = self.R[path]
        return R @ (self.WT @ (self.W @ (R.T @ u))) + self.lam * u

    def _cycle(self, path, r):
        if len(path) == self.L:
            return coarsest_solve(self.leaf[path], r)
        s = self.n >> len(path)
        ops = haar.step_operators_2d(s)
        R = ops["LL"]
        e = R.T @ self._cycle(path + ("LL",), R @ r)
        r2 = r - self.galerkin_apply(path, e)
        for name in self.ORDER[1:]:
            R = ops[name]
            e = e + R.T @ self._cycle(path + (name,), R @ r2)
        return e

    def __call__(self, r):
        return self._cycle((), np.asarray(r, dtype=np.float64).ravel())
