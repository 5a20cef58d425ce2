"""Primal-dual interior point for the conic QP of one time step.

Paper passages followed
-----------------------
* Sec. 2.3: min q(gamma) = 1/2 gamma^T N gamma + r^T gamma subject to
  |(gamma_1, gamma_2)| <= mu gamma_n for every contact.
* Sec. 2.4 ("Primal-Dual Interior Point methods", "The PDIP step",
  "Application to the CCP"): the 2 Nc constraints
  f_i = 1/2 (gamma_1^2 + gamma_2^2 - mu^2 gamma_n^2) and f_{Nc+i} = -gamma_n,
  multipliers lambda_i = -1 / (t f_i), the residual r_t = [grad f0 + Df^T lambda;
  -diag(lambda) f - 1/t] and its Newton system, coupled with a backtracking line
  search and a rule that increases t.
* Sec. 3.3 ("PDIP iteration"): eliminating Delta lambda leaves the 3Nc x 3Nc
  Schur complement S_k = N + M_hat_k - B_k E_k^-1 C_k, symmetric positive
  definite with the sparsity of N (3x3 diagonal blocks added).
* Sec. 3.3 ("Re-using information across timesteps"): start from tangential
  impulses 0 and normal impulse 1, or the previous step's value for a
  persistent contact.

Readings
--------
* The paper names neither the t rule nor the line search; they are those of the
  textbook primal-dual method (Boyd & Vandenberghe, Convex Optimization,
  Sec. 11.7): surrogate gap eta = -f^T lambda, t = mu_pd m / eta with
  mu_pd = 10 and m = 2 Nc; s = 0.99 min(1, min -lambda_i/Dlambda_i), halved
  until the primal point is strictly feasible, then halved until
  |r_t(new)| <= (1 - 0.01 s) |r_t(old)|.
* Multipliers are positive (the paper's "lambda_i < 0" contradicts its own
  lambda_i = -1/(t f_i) with f_i < 0).
* The cone constraint is used in its convex form
  f_i = (gamma_1^2 + gamma_2^2) / (2 mu gamma_n) - mu gamma_n / 2,
  the paper's f_i divided by mu gamma_n > 0.  The feasible set, the number of
  constraints (2 Nc, with f_{Nc+i} = -gamma_n) and the QP are unchanged.  The
  textbook method assumes convex f_i; the paper's quadratic form is not convex
  and its gradient vanishes at the apex of the cone, where every separating
  contact's optimum lies, so its multiplier must diverge there and the
  residual line search stalls (on a 216-sphere box the dual residual stays
  near 1 after 400 iterations).  In the convex form the multipliers stay
  bounded and the same method reaches a gap of 1e-8 in about 30 iterations.
* Eliminating Delta lambda exactly gives the 3x3 blocks
  H_i = lambda_i hess f_i + lambda_i/(-f_i) g_i g_i^T
        + lambda_{Nc+i}/gamma_n e_n e_n^T,   g_i = grad f_i,
  the diagonal blocks that Sec. 3.3 adds to N (its diagonal M_hat plus the
  block-diagonal B E^-1 C).
* Schur right-hand side (derived from the Newton system; the paper prints it
  not): rhs = -(N gamma + r) + (1/t) sum_i grad f_i / f_i.
* Stopping: eta / m <= tol_gap (1e-8) and |r_dual|_inf <= tol_dual (1e-4), in
  scaled units (impulses over m_bar g h, velocities over g h).  The dual
  residual of separating contacts decays only linearly once the gap is small,
  so its tolerance is looser than the gap's.
* Start: lambda^0_i = 1 / (t0 (-f_i(gamma^0))) with t0 = 1 (on the central path
  of t = 1 for the constraint part).
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclasses.dataclass
class PdipParams:
    mu_pd: float = 10.0
    alpha: float = 0.01
    beta: float = 0.5
    tol_gap: float = 1e-8
    tol_dual: float = 1e-4
    maxit: int = 100
    max_backtrack: int = 80


def _split(gamma):
    g = gamma.reshape(-1, 3)
    return g[:, 0], g[:, 1], g[:, 2]


def constraints(gamma, mu):
    """f in R^{2 Nc}: cone constraints (convex form) first, then -gamma_n."""
    gn, g1, g2 = _split(gamma)
    f1 = (g1 * g1 + g2 * g2) / (2.0 * mu * gn) - 0.5 * mu * gn
    return np.concatenate([f1, -gn])


def cone_gradient(gamma, mu):
    """grad f_i of the cone constraints, [Nc][3]."""
    gn, g1, g2 = _split(gamma)
    t2 = g1 * g1 + g2 * g2
    return np.stack([-t2 / (2.0 * mu * gn * gn) - 0.5 * mu,
                     g1 / (mu * gn), g2 / (mu * gn)], axis=1)


def cone_hessian(gamma, mu):
    """hess f_i of the cone constraints, [Nc][3][3]."""
    gn, g1, g2 = _split(gamma)
    t2 = g1 * g1 + g2 * g2
    H = np.zeros((gn.size, 3, 3))
    H[:, 0, 0] = t2 / (mu * gn ** 3)
    H[:, 0, 1] = H[:, 1, 0] = -g1 / (mu * gn * gn)
    H[:, 0, 2] = H[:, 2, 0] = -g2 / (mu * gn * gn)
    H[:, 1, 1] = H[:, 2, 2] = 1.0 / (mu * gn)
    return H


def constraint_jacobian(gamma, mu):
    """Df (2Nc x 3Nc), sparse."""
    G = cone_gradient(gamma, mu)
    nc = G.shape[0]
    i = np.arange(nc)
    rows = np.concatenate([i, i, i, nc + i])
    cols = np.concatenate([3 * i, 3 * i + 1, 3 * i + 2, 3 * i])
    vals = np.concatenate([G[:, 0], G[:, 1], G[:, 2], -np.ones(nc)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * nc, 3 * nc))


def residuals(N, r, gamma, lam, mu, t):
    """r_dual = N gamma + r + Df^T lambda and r_cent = -lambda f - 1/t."""
    f = constraints(gamma, mu)
    J = constraint_jacobian(gamma, mu)
    r_dual = N @ gamma + r + J.T @ lam
    r_cent = -lam * f - 1.0 / t
    return r_dual, r_cent


def barrier_blocks(gamma, lam, mu):
    """The 3x3 blocks H_i added to N on the diagonal (see module readings)."""
    gn = gamma.reshape(-1, 3)[:, 0]
    nc = gn.size
    f = constraints(gamma, mu)
    f1, lam1, lam2 = f[:nc], lam[:nc], lam[nc:]
    grad = cone_gradient(gamma, mu)
    H = lam1[:, None, None] * cone_hessian(gamma, mu)
    H += (lam1 / (-f1))[:, None, None] * grad[:, :, None] * grad[:, None, :]
    H[:, 0, 0] += lam2 / gn
    return H


def schur_matrix(N, gamma, lam, mu):
    """S = N + blockdiag(H_i) (Sec. 3.3)."""
    H = barrier_blocks(gamma, lam, mu)
    return (N + sp.block_diag(list(H), format="csr")).tocsr()


def schur_rhs(N, r, gamma, mu, t):
    """-(N gamma + r) + (1/t) Df^T (1 / f)."""
    f = constraints(gamma, mu)
    J = constraint_jacobian(gamma, mu)
    return -(N @ gamma + r) + (1.0 / t) * (J.T @ (1.0 / f))


def back_substitute(gamma, lam, mu, t, dgamma):
    """Delta lambda from the second block row of the Newton system."""
    f = constraints(gamma, mu)
    J = constraint_jacobian(gamma, mu)
    r_cent = -lam * f - 1.0 / t
    return (r_cent - lam * (J @ dgamma)) / f


def unreduced_system(N, r, gamma, lam, mu, t):
    """The full (3Nc + 2Nc) Newton system of Sec. 2.4 and its right-hand side."""
    nc = gamma.size // 3
    f = constraints(gamma, mu)
    J = constraint_jacobian(gamma, mu)
    hess = sp.block_diag(list(lam[:nc, None, None] * cone_hessian(gamma, mu)),
                         format="csr")
    A = sp.bmat([[N + hess, J.T],
                 [-sp.diags(lam) @ J, -sp.diags(f)]], format="csc")
    r_dual, r_cent = residuals(N, r, gamma, lam, mu, t)
    return A, -np.concatenate([r_dual, r_cent])


def direct_solve(S, rhs):
    """Sparse direct Newton-step solve: dense Cholesky when small, else SuperLU."""
    n = S.shape[0]
    if n <= 3000:
        c = sla.cho_factor(S.toarray())
        return sla.cho_solve(c, rhs)
    lu = spla.splu(sp.csc_matrix(S), permc_spec="MMD_AT_PLUS_A")
    return lu.solve(rhs)


@dataclasses.dataclass
class PdipResult:
    gamma: np.ndarray
    lam: np.ndarray
    iterations: int
    converged: bool
    gap: float
    dual_inf: float
    history: list


def initial_point(nc, mu, gamma_n0=None, t0=1.0):
    gamma = np.zeros(3 * nc)
    gamma[0::3] = 1.0 if gamma_n0 is None else gamma_n0
    f = constraints(gamma, mu)
    lam = 1.0 / (t0 * (-f))
    return gamma, lam


def pdip(N, r, mu, params=None, gamma0=None, lam0=None, solve=None,
         record=False):
    """Primal-dual interior point method (Sec. 2.4; B&V Sec. 11.7 steps).

    N, r in scaled units.  ``solve(S, rhs)`` returns the Newton step (default:
    sparse direct).  With ``record`` the history keeps, per iteration, the
    Schur matrix, its right-hand side and the step, for parity checks.
    """
    p = params or PdipParams()
    solve = solve or direct_solve
    nc = r.size // 3
    m = 2 * nc
    if gamma0 is None:
        gamma, lam = initial_point(nc, mu)
    else:
        gamma = gamma0.copy()
        lam = lam0.copy() if lam0 is not None else 1.0 / (-constraints(gamma, mu))
    hist = []
    converged = False
    it = 0
    gap = dual_inf = np.inf
    while True:
        f = constraints(gamma, mu)
        gap = float(-f @ lam)
        # B&V's rule t = mu m / eta, capped where the central point already
        # meets the gap tolerance: further increase only worsens the
        # conditioning of S while the dual residual is being driven down
        t = min(p.mu_pd * m / gap, p.mu_pd / p.tol_gap)
        r_dual, r_cent = residuals(N, r, gamma, lam, mu, t)
        dual_inf = float(np.abs(r_dual).max()) if nc else 0.0
        if gap / m <= p.tol_gap and dual_inf <= p.tol_dual:
            converged = True
            break
        if it >= p.maxit:
            break
        S = schur_matrix(N, gamma, lam, mu)
        rhs = schur_rhs(N, r, gamma, mu, t)
        dgamma = solve(S, rhs)
        dlam = back_substitute(gamma, lam, mu, t, dgamma)
        # line search (B&V Sec. 11.7.3)
        neg = dlam < 0
        s_max = min(1.0, float(np.min(-lam[neg] / dlam[neg]))) if neg.any() else 1.0
        s = 0.99 * s_max
        nb = 0
        while np.any(constraints(gamma + s * dgamma, mu) >= 0.0):
            s *= p.beta
            nb += 1
            if nb > p.max_backtrack:
                raise RuntimeError("line search: no strictly feasible step")
        norm0 = np.sqrt(r_dual @ r_dual + r_cent @ r_cent)
        while True:
            rd, rc = residuals(N, r, gamma + s * dgamma, lam + s * dlam, mu, t)
            if np.sqrt(rd @ rd + rc @ rc) <= (1.0 - p.alpha * s) * norm0:
                break
            s *= p.beta
            nb += 1
            if nb > p.max_backtrack:
                break
        if record:
            hist.append(dict(S=S, rhs=rhs, dgamma=dgamma, dlam=dlam, t=t,
                             gap=gap, step=s, gamma=gamma.copy(),
                             lam=lam.copy()))
        else:
            hist.append(dict(t=t, gap=gap, step=s, dual_inf=dual_inf))
        gamma = gamma + s * dgamma
        lam = lam + s * dlam
        it += 1
    return PdipResult(gamma, lam, it, converged, gap, dual_inf, hist)


def time_step(scene, params=None, contacts=None, record=False, gamma_n0=None):
    """Detect, assemble, solve the QP with PDIP and integrate one step.

    Returns (contacts, result, gamma_physical, (x, v, w)).
    """
    from . import assembly, contacts as ct
    c = contacts if contacts is not None else ct.detect(scene)
    N, r, D = assembly.qp_data(scene, c)
    gbar, vbar = assembly.scales(scene)
    mbar = gbar / vbar
    Ns = (N * mbar).tocsr()
    rs = r / vbar
    g0 = l0 = None
    if gamma_n0 is not None:
        g0, l0 = initial_point(c.nc, scene.mu, gamma_n0)
    res = pdip(Ns, rs, scene.mu, params, gamma0=g0, lam0=l0, record=record)
    gamma = res.gamma * gbar
    new_state = assembly.integrate(scene, D, gamma)
    return c, res, gamma, new_state
