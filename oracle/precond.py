"""The QTT preconditioner of the Newton-step solve, dense and plain.

Paper passages followed
-----------------------
* Sec. 3.3 ("TT Newton system solver"): tensorise the Schur complement on the
  contact hierarchy, build TT approximations of the matrix and of its inverse
  at a target accuracy, and use the inverse directly or as the preconditioner
  of a Krylov method; hot-start the next approximations from the current ones
  (S_{k+1} = S_k + L_k with L_k block-diagonal).
* Sec. 3.1 Algorithm 1 (compression), Sec. 3.2 (inverse updates).

Readings
--------
* The matrix compressed is the block-Jacobi scaled S~ = L^-1 S L^-T with
  L = blockdiag(chol S_ss) over contact slots (dummy slots: identity), so that
  every 3x3 diagonal block is the identity; the preconditioner is
  P = L^-T X L^-1 with X ~ S~^-1.
* Algorithm 1 is run from the last mode to the first (tt.tt_svd_reversed):
  its first truncations act on the finest blocks, where the sparse matrix
  lives, with the same per-bond tolerance eps |S~|_F / sqrt(d-1) and a rank
  cap rmax_s.
* The inverse is built by Newton-Schulz, X0 = I / |S~|_inf (max absolute row
  sum of the exact S~), Y = round(S~_TT X) with cap rmax_s,
  X <- round(2 X - X Y) with cap rmax.  After each iteration the probe
  residual max over z of rms(z - S~ X z) with the exact S~ and the two fixed
  probes z1 = 1, z2_i = (-1)^popcount(i) is evaluated; iteration stops when it
  does not decrease, and the iterate with the smallest probe residual is kept.
"""

from __future__ import annotations

import numpy as np

from . import tt


def block_jacobi_inverse_factors(S):
    """Dense L^-1 for the 3x3 block Cholesky factors of S (n = 2^d, padded)."""
    n = S.shape[0]
    Linv = np.eye(n)
    for s in range(n // 3):
        b = slice(3 * s, 3 * s + 3)
        Linv[b, b] = np.linalg.inv(np.linalg.cholesky(S[b, b]))
    return Linv


def scaled_matrix(S):
    Linv = block_jacobi_inverse_factors(S)
    return Linv @ S @ Linv.T, Linv


def probes(n):
    i = np.arange(n, dtype=np.uint64)
    pc = np.zeros(n, dtype=np.int64)
    v = i.copy()
    while np.any(v):
        pc += (v & np.uint64(1)).astype(np.int64)
        v >>= np.uint64(1)
    return np.ones(n), np.where(pc % 2 == 1, -1.0, 1.0)


def probe_residual(St, X_dense):
    worst = 0.0
    n = St.shape[0]
    for z in probes(n):
        r = z - St @ (X_dense @ z)
        worst = max(worst, float(np.sqrt(r @ r / n)))
    return worst


def build_inverse(St, eps, rmax_s, rmax, iters, X0=None):
    """Compression of S~ and Newton-Schulz inverse with the probe rule.

    Returns (A_cores, X_cores, iterations_done, best_probe).
    """
    d = int(round(np.log2(St.shape[0])))
    A = tt.qtt_from_dense_reversed(St, eps, rmax_s)
    if X0 is None:
        X = tt.qtt_scale(tt.qtt_identity(d), 1.0 / np.abs(St).sum(axis=1).max())
    else:
        X = X0
    best = probe_residual(St, tt.qtt_to_dense(X))
    bestX = X
    done = 0
    for _ in range(iters):
        Y = tt.tt_round(tt.qtt_matmul(A, X), eps, rmax_s)
        T = tt.qtt_add(tt.qtt_scale(X, 2.0), tt.qtt_scale(tt.qtt_matmul(X, Y), -1.0))
        X = tt.tt_round(T, eps, rmax)
        done += 1
        pr = probe_residual(St, tt.qtt_to_dense(X))
        if not pr < best:
            break
        best = pr
        bestX = X
    return A, bestX, done, best
