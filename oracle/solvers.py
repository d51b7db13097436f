"""Krylov and SIRT solvers on the tomographic normal equations (oracle, float64).

All solvers start from x0 = 0 (the paper's error definitions ||e_k||/||e_0|| and
||x_k - x_ex||/||x_ex|| in Tables 1 and 2 coincide only then).

PCGLS (CGLS, a Krylov method of Section 2.3.1, with a symmetric positive
definite M^-1 applied to the normal equations K x = W^T b, K = W^T W + lam I, eq. sys_ne / sys_reg):
    x = 0, r = b, s = W^T r - lam x, z = M^-1 s, p = z, gamma = <s, z>
    repeat:
        q = W p;  delta = ||q||^2 + lam ||p||^2;  alpha = gamma / delta
        x += alpha p;  r -= alpha q
        s = W^T r - lam x;  z = M^-1 s
        gamma' = <s, z>;  beta = gamma'/gamma;  p = z + beta p
        relres = ||s|| / ||s_0||
The relative residual is that of the solved normal equations (the paper plots
||r_k||/||r_0|| of the system Krylov solves, Section 4.1).

GMRES(restart), right preconditioned (eq. sys_prec, second form): solve
K M^-1 u = f with f = W^T b, x = M^-1 u, Arnoldi with modified Gram-Schmidt and
Givens rotations; residual estimate |g_{j+1}| / ||f||.  One matvec = one W and
one W^T application.

BiCGStab, right preconditioned (the paper's primary Krylov solver, Section
2.3.1, on the normal equations with A = W^T W (+ lam I) and f = W^T b, right
preconditioning as in eq. sys_prec): van der Vorst's recursion with shadow
vector rhat = r_0 = f, x_0 = 0,
    rho = <rhat, r>;  beta = (rho / rho_prev) (alpha / omega)
    p = r + beta (p - omega v);  phat = M^-1 p;  v = K phat
    alpha = rho / <rhat, v>;  s = r - alpha v
    shat = M^-1 s;  t = K shat;  omega = <t, s> / <t, t>   (0 when t = 0)
    x += alpha phat + omega shat;  r = s - omega t
relres = ||r|| / ||r_0||; two matvecs per iteration.  The paper does not give
the variant: this is the textbook one (reading listed in the design notes).

SIRT (eq. sys_sirt, eq. sirt_it): R = inverse row sums, C = inverse column
sums (0 where a sum is 0), x <- x + C W^T R (b - W x); relres is
||C W^T R (b - W x_k)|| / ||C W^T R b||.

Parity status: PCGLS pinned by the Krylov-subspace minimisation property and
dense least squares on tiny systems; GMRES by brute-force minimisation over
the Krylov space and exact solve with restart >= N; BiCGStab by the step
properties (<rhat, s> = 0, r orthogonal to t), the recursive residual equal
to the true one, convergence to the dense solve and a one-step solve with the
exact preconditioner; SIRT by the closed form x_k = sum_{i<k} S^i C W^T R b.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Result:
    x: np.ndarray
    iters: int
    matvecs: int
    relres: float
    history: list = field(default_factory=list)
    converged: bool = False


def _identity(v):
    return v


def pcgls(W, b, tol=1e-3, max_iter=1000, lam=0.0, precond=None, fixed_iters=None,
          callback=None, store=None) -> Result:
    """Preconditioned CGLS.  fixed_iters runs exactly that many iterations.

    store, if given, is applied to every vector the recursion keeps (x, r, p,
    q, s, z) right after it is formed; tests use it to model a lower storage
    precision.  It is the identity otherwise."""
    Minv = precond or _identity
    hook = store or _identity
    b = np.asarray(b, dtype=np.float64).ravel()
    x = np.zeros(W.shape[1])
    r = hook(b.copy())
    s = hook(W.T @ r - lam * x)
    z = hook(Minv(s))
    p = z.copy()
    gamma = float(s @ z)
    s0 = float(np.linalg.norm(s))
    hist = []
    if s0 == 0.0:
        return Result(x, 0, 1, 0.0, hist, True)
    k = 0
    limit = fixed_iters if fixed_iters is not None else max_iter
    converged = False
    relres = 1.0
    while k < limit:
        q = hook(W @ p)
        delta = float(q @ q) + lam * float(p @ p)
        alpha = gamma / delta
        x = hook(x + alpha * p)
        r = hook(r - alpha * q)
        s = hook(W.T @ r - lam * x)
        z = hook(Minv(s))
        gamma_new = float(s @ z)
        beta = gamma_new / gamma
        gamma = gamma_new
        p = hook(z + beta * p)
        k += 1
        relres = float(np.linalg.norm(s)) / s0
        hist.append(relres)
        if callback is not None:
            callback(k, x)
        if fixed_iters is None and relres <= tol:
            converged = True
            break
    return Result(x, k, 1 + k, relres, hist, converged)


def gmres_right(W, b, tol=1e-3, restart=30, max_iter=1000, lam=0.0, precond=None,
                fixed_iters=None, store=None) -> Result:
    """Right-preconditioned restarted GMRES on (W^T W + lam I) M^-1 u = W^T b.

    store, if given, is applied to every stored vector (basis vectors, the
    new Krylov vector, x) right after it is formed; tests use it to model a
    lower storage precision.  It is the identity otherwise."""
    Minv = precond or _identity
    hook = store or _identity

    def K(v):
        return W.T @ (W @ v) + lam * v

    b = np.asarray(b, dtype=np.float64).ravel()
    N = W.shape[1]
    f = W.T @ b
    fnorm = float(np.linalg.norm(f))
    x = np.zeros(N)
    hist = []
    if fnorm == 0.0:
        return Result(x, 0, 0, 0.0, hist, True)
    limit = fixed_iters if fixed_iters is not None else max_iter
    total = 0
    matvecs = 0
    relres = 1.0
    converged = False
    r = f.copy()
    while total < limit and not converged:
        beta = float(np.linalg.norm(r))
        V = np.zeros((restart + 1, N))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = hook(r / beta)
        j_done = 0
        for j in range(restart):
            w = hook(K(Minv(V[j])))
            matvecs += 1
            for i in range(j + 1):           # modified Gram-Schmidt
                H[i, j] = float(V[i] @ w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] != 0.0:
                V[j + 1] = hook(w / H[j + 1, j])
            for i in range(j):               # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            relres = abs(g[j + 1]) / fnorm
            hist.append(relres)
            if fixed_iters is None and relres <= tol:
                converged = True
                break
            if total >= limit:
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):      # back substitution
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:j_done]) / H[i, i]
        x = hook(x + Minv(V[:j_done].T @ y))
        if not converged and total < limit:
            r = f - K(x)                          # true residual at restart
            matvecs += 1
    return Result(x, total, matvecs, relres, hist, converged)


def bicgstab_right(W, b, tol=1e-3, max_iter=1000, lam=0.0, precond=None, fixed_iters=None,
                   callback=None) -> Result:
    """Right-preconditioned BiCGStab on (W^T W + lam I) M^-1 u = W^T b, x = M^-1 u.

    Stops when ||r|| / ||r_0|| <= tol (not with fixed_iters), after max_iter
    iterations, or at a breakdown (rho = 0 or <rhat, v> = 0; converged stays
    False).  callback(i, vectors), if given, receives after iteration i a dict
    of that iteration's rhat, r_prev, p, phat, v, s, shat, t, x, r and the
    scalars alpha, omega, rho."""
    Minv = precond or _identity

    def K(v):
        return W.T @ (W @ v) + lam * v

    b = np.asarray(b, dtype=np.float64).ravel()
    N = W.shape[1]
    f = W.T @ b
    r = f.copy()
    r0norm = float(np.linalg.norm(r))
    x = np.zeros(N)
    hist = []
    if r0norm == 0.0:
        return Result(x, 0, 0, 0.0, hist, True)
    rhat = r.copy()
    p = np.zeros(N)
    v = np.zeros(N)
    rho_prev = alpha = omega = 1.0
    limit = fixed_iters if fixed_iters is not None else max_iter
    relres = 1.0
    converged = False
    it = 0
    while it < limit:
        rho = float(rhat @ r)
        if rho == 0.0 or not np.isfinite(rho):
            break
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        phat = Minv(p)
        v = K(phat)
        rv = float(rhat @ v)
        if rv == 0.0 or not np.isfinite(rv):
            break
        alpha = rho / rv
        s = r - alpha * v
        shat = Minv(s)
        t = K(shat)
        tt = float(t @ t)
        omega = float(t @ s) / tt if tt != 0.0 else 0.0
        r_prev = r
        x = x + alpha * phat + omega * shat
        r = s - omega * t
        rho_prev = rho
        it += 1
        relres = float(np.linalg.norm(r)) / r0norm
        hist.append(relres)
        if callback is not None:
            callback(it, dict(rhat=rhat, r_prev=r_prev, p=p, phat=phat, v=v, s=s, shat=shat, t=t,
                              x=x, r=r, alpha=alpha, omega=omega, rho=rho))
        if fixed_iters is None and relres <= tol:
            converged = True
            break
        if omega == 0.0:
            break
    return Result(x, it, 2 * it, relres, hist, converged)


def sirt_weights(W):
    """(R, C): inverse row and column sums of W, 0 where the sum is 0."""
    rs = np.asarray(W.sum(axis=1)).ravel()
    cs = np.asarray(W.sum(axis=0)).ravel()
    R = np.zeros_like(rs)
    C = np.zeros_like(cs)
    R[rs != 0] = 1.0 / rs[rs != 0]
    C[cs != 0] = 1.0 / cs[cs != 0]
    return R, C


def sirt(W, b, tol=1e-3, max_iter=1000, fixed_iters=None) -> Result:
    """SIRT, x_{k+1} = x_k + C W^T R (b - W x_k) from x_0 = 0."""
    b = np.asarray(b, dtype=np.float64).ravel()
    R, C = sirt_weights(W)
    x = np.zeros(W.shape[1])
    ref = float(np.linalg.norm(C * (W.T @ (R * b))))
    hist = []
    if ref == 0.0:
        return Result(x, 0, 0, 0.0, hist, True)
    limit = fixed_iters if fixed_iters is not None else max_iter
    k = 0
    converged = False
    relres = 1.0
    while k < limit:
        upd = C * (W.T @ (R * (b - W @ x)))
        relres = float(np.linalg.norm(upd)) / ref
        x = x + upd
        k += 1
        hist.append(relres)
        if fixed_iters is None and relres <= tol:
            converged = True
            break
    return Result(x, k, k, relres, hist, converged)
