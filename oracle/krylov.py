"""Flexible GMRES with right preconditioning (Saad, SIAM J. Sci. Comput. 1993).

The paper solves the Newton system either directly with the approximate TT
inverse or with a preconditioned Krylov method (Sec. 3.3, "TT Newton system
solver"; Sec. 4.2 uses BiCGSTAB).  The GPU path uses flexible GMRES because it
tolerates a preconditioner that changes or is applied in reduced precision.

Plain restarted FGMRES(m): Arnoldi with classical Gram-Schmidt applied twice,
Givens rotations on the Hessenberg matrix, the residual estimate |g_{j+1}|,
and x = x0 + Z y on convergence or at restart.
"""

from __future__ import annotations

import numpy as np


def fgmres(matvec, precond, b, x0=None, tol=1e-8, restart=30, maxit=1000):
    """Solve A x = b to |b - A x| <= tol |b|; returns (x, iterations, history)."""
    n = b.size
    x = np.zeros(n) if x0 is None else x0.copy()
    bnorm = float(np.linalg.norm(b))
    hist = []
    if bnorm == 0.0:
        return np.zeros(n), 0, hist
    it = 0
    while it < maxit:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        hist.append(beta / bnorm)
        if beta <= tol * bnorm:
            break
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            h1 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h1
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            H[:j + 1, j] = h1 + h2
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # apply previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + Z[:j_end].T @ y
        if abs(g[j_end]) <= tol * bnorm:
            # confirm with the true residual on the next pass
            r = b - matvec(x)
            if np.linalg.norm(r) <= tol * bnorm:
                break
    return x, it, hist
