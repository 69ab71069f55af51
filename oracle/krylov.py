"""Right-preconditioned FGMRES and GMRES (oracle).

The paper uses GMRES with the (linear) two-grid sweeping preconditioner
(Sec. 1 and Sec. 4) and stops when the residual is reduced by 1e-6
(Sec. 5, implementation).  Here: x0 = 0, modified Gram-Schmidt Arnoldi, Givens rotations,
stop when the Arnoldi residual estimate <= tol * ||b||, restart after
``restart`` inner steps.  FGMRES stores z_j = M v_j and forms x = Z y; GMRES
forms x = M (V y).  For a fixed linear M both give the same iterates.
"""
from __future__ import annotations

import numpy as np


def _givens(a, b):
    """Rotation [[c, s], [-conj(s), c]] with real c that zeroes b below a."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, 1.0
    t = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def fgmres(matvec, precond, b, tol=1e-6, maxit=200, restart=None, flexible=True,
           callback=None):
    """Solve A x = b.  Returns (x, iterations, residual-estimate history,
    true relative residual).  ``callback(k, x_k)`` (optional) is called with
    the k-th iterate (k = 1, 2, ...) - this forms x_k explicitly each step
    and is meant for tests only."""
    b = np.asarray(b, dtype=complex).ravel()
    n = b.size
    restart = maxit if restart is None else restart
    x = np.zeros(n, dtype=complex)
    bnorm = np.linalg.norm(b)
    hist = [1.0]
    if bnorm == 0:
        return x, 0, hist, 0.0
    it = 0
    while it < maxit:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        m = min(restart, maxit - it)
        V = np.zeros((m + 1, n), dtype=complex)
        Z = np.zeros((m, n), dtype=complex) if flexible else None
        H = np.zeros((m + 1, m), dtype=complex)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=complex)
        g = np.zeros(m + 1, dtype=complex)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        done = False
        for k in range(m):
            z = precond(V[k])
            if flexible:
                Z[k] = z
            w = matvec(z)
            for i in range(k + 1):
                H[i, k] = np.vdot(V[i], w)
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -np.conj(sn[i]) * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            cs[k], sn[k] = _givens(H[k, k], H[k + 1, k])
            H[k, k] = cs[k] * H[k, k] + sn[k] * H[k + 1, k]
            H[k + 1, k] = 0.0
            g[k + 1] = -np.conj(sn[k]) * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_used = k + 1
            hist.append(abs(g[k + 1]) / bnorm)
            if callback is not None:
                y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
                xk = x + (y @ Z[:k_used] if flexible else precond(y @ V[:k_used]))
                callback(it, xk)
            if abs(g[k + 1]) <= tol * bnorm:
                done = True
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        if flexible:
            x = x + y @ Z[:k_used]
        else:
            x = x + precond(y @ V[:k_used])
        if done:
            break
    relres = np.linalg.norm(b - matvec(x)) / bnorm
    return x, it, hist, relres
