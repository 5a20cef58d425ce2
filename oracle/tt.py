"""Tensor-train (TT) and quantized tensor-train (QTT) toolkit, dense and plain.

Paper passages followed
-----------------------
* Sec. 3.1: index convention i = (i_1 i_2 ... i_d), lexicographic with i_1 the
  most significant; TT decomposition A(i_1..i_d) = G_1(i_1) G_2(i_2) ... G_d(i_d)
  with cores G_k(alpha_{k-1}, i_k, alpha_k); unfolding matrices; the TT ranks
  are the ranks of the unfoldings.
* Sec. 3.1, Algorithm 1 (TT decomposition): a left-to-right chain of low-rank
  approximations of the unfoldings, each to accuracy eps / sqrt(d-1).
* Sec. 3.2: a matrix of size 2^d is tensorised on the product of binary trees,
  A_T(b_1..b_d) = A(i_1..i_d, j_1..j_d) with b_k = (i_k, j_k); each core is a
  2x2 matrix parametrised by (alpha_{k-1}, alpha_k); the TT matrix-vector
  product contracts one dimension at a time.

Readings
--------
* The per-step tolerance of Algorithm 1 is relative: each truncation discards
  singular values whose squared sum is at most (eps |A|_F)^2 / (d-1), so that
  |A - A_TT|_F <= eps |A|_F.
* Inside a QTT core the mode index is b_k = 2 i_k + j_k (row bit first); cores
  are stored as arrays [r_{k-1}, 2, 2, r_k] indexed (alpha, i_k, j_k, beta).
* Rounding (re-compression of a TT with redundant ranks) is the standard
  orthogonalise-then-truncate procedure (Oseledets, "Tensor-Train
  Decomposition", SIAM J. Sci. Comput. 2011): right-to-left QR, then a
  left-to-right truncated SVD with the same per-bond tolerance as Algorithm 1.
* The approximate inverse is built by the Newton-Schulz iteration
  X <- X (2 I - A X) with rounding after each product (the paper inverts by
  ALS; see the inverse-update paragraph of Sec. 3.2).
"""

from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------
# plain TT of a dense tensor (Algorithm 1)
# ----------------------------------------------------------------------------

def truncation_rank(s, delta, rmax=None):
    """Smallest r with sum_{l > r} s_l^2 <= delta^2 (at least 1), capped at rmax."""
    tail = np.cumsum((s ** 2)[::-1])[::-1]  # tail[l] = sum_{q >= l} s_q^2
    r = len(s)
    for l in range(1, len(s) + 1):
        if l == len(s) or tail[l] <= delta * delta:
            r = l
            break
    r = max(r, 1)
    if rmax is not None:
        r = min(r, rmax)
    return r


def tt_svd(A, eps, rmax=None):
    """Algorithm 1: TT cores of the dense tensor A (shape n_1 x ... x n_d).

    Each unfolding M_k is approximated by a truncated SVD U_k S_k V_k^T; the
    left factor U_k is the k-th core and S_k V_k^T, reshaped, is M_{k+1}.
    """
    shape = A.shape
    d = len(shape)
    delta = eps * np.linalg.norm(A.ravel()) / np.sqrt(max(d - 1, 1))
    cores = []
    r_prev = 1
    Mk = A.reshape(shape[0], -1)
    for k in range(d - 1):
        U, s, Vt = np.linalg.svd(Mk, full_matrices=False)
        rk = truncation_rank(s, delta, rmax)
        cores.append(U[:, :rk].reshape(r_prev, shape[k], rk))
        Vk = s[:rk, None] * Vt[:rk, :]
        Mk = Vk.reshape(rk * shape[k + 1], -1)
        r_prev = rk
    cores.append(Mk.reshape(r_prev, shape[d - 1], 1))
    return cores


def tt_full(cores):
    """Dense tensor from TT cores (contract the chain)."""
    T = cores[0]  # [1, n1, r1]
    for G in cores[1:]:
        T = np.tensordot(T, G, axes=([T.ndim - 1], [0]))
    return T.reshape([G.shape[1] for G in cores])


def tt_ranks(cores):
    return [int(G.shape[2]) for G in cores[:-1]]


def unfolding_singular_values(A, k):
    """Singular values of the k-th unfolding of a dense tensor (1-based k)."""
    n = A.shape
    return np.linalg.svd(A.reshape(int(np.prod(n[:k])), -1), compute_uv=False)


# ----------------------------------------------------------------------------
# QTT matrices
# ----------------------------------------------------------------------------

def qtt_tensorize(A):
    """N x N matrix (N = 2^d) -> d-way tensor with modes b_k = 2 i_k + j_k."""
    N = A.shape[0]
    d = int(round(np.log2(N)))
    assert 1 << d == N and A.shape == (N, N)
    T = A.reshape([2] * d + [2] * d)
    perm = []
    for k in range(d):
        perm += [k, d + k]
    return T.transpose(perm).reshape([4] * d)


def qtt_untensorize(T):
    d = T.ndim
    T = T.reshape([2, 2] * d)
    perm = [2 * k for k in range(d)] + [2 * k + 1 for k in range(d)]
    return T.transpose(perm).reshape(1 << d, 1 << d)


def qtt_from_dense(A, eps, rmax=None):
    """QTT cores [r, 2, 2, r'] of a dense matrix by Algorithm 1."""
    cores = tt_svd(qtt_tensorize(A), eps, rmax)
    return [G.reshape(G.shape[0], 2, 2, G.shape[2]) for G in cores]


def qtt_to_dense(cores):
    flat = [G.reshape(G.shape[0], 4, G.shape[3]) for G in cores]
    return qtt_untensorize(tt_full(flat))


def qtt_entry(cores, i, j):
    """A(i, j) as a product of d small matrices (works for any d)."""
    d = len(cores)
    v = np.ones((1,))
    for k in range(d):
        ik = (i >> (d - 1 - k)) & 1
        jk = (j >> (d - 1 - k)) & 1
        v = v @ cores[k][:, ik, jk, :]
    return float(v[0])


def qtt_matvec(cores, x):
    """y = A x contracting one dimension at a time (Sec. 3.2).

    Z_0 = x viewed as [1][j_1..j_d]; step k replaces (alpha_{k-1}, j_k) by
    (i_k, alpha_k): Z_k[I, i_k, alpha_k, J] = sum G_k(alpha, i_k, j_k, beta)
    Z_{k-1}[I, alpha, j_k, J].
    """
    d = len(cores)
    N = 1 << d
    Z = np.asarray(x, dtype=np.float64).reshape(1, 1, N)  # [I][alpha][J]
    for k, G in enumerate(cores):
        P, ra, rest = Z.shape
        Z = Z.reshape(P, ra, 2, rest // 2)
        Z = np.einsum("aijb,pajr->pibr", G, Z)
        Z = Z.reshape(P * 2, G.shape[3], rest // 2)
    return Z.reshape(N)


def qtt_identity(d):
    return [np.eye(2).reshape(1, 2, 2, 1).copy() for _ in range(d)]


def qtt_scale(cores, a):
    out = [G.copy() for G in cores]
    out[0] = out[0] * a
    return out


def qtt_add(A, B):
    """Cores of A + B (ranks add): block-diagonal middle cores."""
    d = len(A)
    out = []
    for k in range(d):
        a, b = A[k], B[k]
        if k == 0:
            out.append(np.concatenate([a, b], axis=3))
        elif k == d - 1:
            out.append(np.concatenate([a, b], axis=0))
        else:
            G = np.zeros((a.shape[0] + b.shape[0], 2, 2, a.shape[3] + b.shape[3]))
            G[:a.shape[0], :, :, :a.shape[3]] = a
            G[a.shape[0]:, :, :, a.shape[3]:] = b
            out.append(G)
    return out


def qtt_matmul(A, B):
    """Cores of the matrix product A B: C_k = sum_l A_k(., i, l, .) B_k(., l, j, .)."""
    out = []
    for a, b in zip(A, B):
        C = np.einsum("pilq,sljt->psijqt", a, b)
        out.append(C.reshape(a.shape[0] * b.shape[0], 2, 2,
                             a.shape[3] * b.shape[3]))
    return out


def qtt_norm(cores):
    return float(np.linalg.norm(qtt_to_dense(cores)))


def tt_round(cores, eps, rmax=None, shape4=True):
    """TT rounding: right-to-left QR, then left-to-right truncated SVD.

    Tolerance per bond eps |A|_F / sqrt(d-1), rank cap rmax.
    """
    d = len(cores)
    G = [c.reshape(c.shape[0], -1, c.shape[-1]).copy() for c in cores]
    n = [g.shape[1] for g in G]
    # right-to-left orthogonalisation: cores 2..d become right-orthonormal
    for k in range(d - 1, 0, -1):
        r0, nk, r1 = G[k].shape
        Q, R = np.linalg.qr(G[k].reshape(r0, nk * r1).T)
        G[k] = Q.T.reshape(-1, nk, r1)
        G[k - 1] = np.tensordot(G[k - 1], R.T, axes=([2], [0]))
    nrm = np.linalg.norm(G[0].ravel())
    delta = eps * nrm / np.sqrt(max(d - 1, 1))
    for k in range(d - 1):
        r0, nk, r1 = G[k].shape
        U, s, Vt = np.linalg.svd(G[k].reshape(r0 * nk, r1), full_matrices=False)
        rk = truncation_rank(s, delta, rmax)
        G[k] = U[:, :rk].reshape(r0, nk, rk)
        G[k + 1] = np.tensordot(s[:rk, None] * Vt[:rk, :], G[k + 1],
                                axes=([1], [0]))
    if shape4:
        return [g.reshape(g.shape[0], 2, 2, g.shape[2]) for g in G]
    return G


def newton_schulz(A, X0, eps, rmax, iters):
    """Newton-Schulz X <- round(2X - X round(A X)) in QTT form.

    Returns the list of iterates (X0 excluded).
    """
    X = X0
    out = []
    for _ in range(iters):
        Y = tt_round(qtt_matmul(A, X), eps, rmax)
        XY = qtt_matmul(X, Y)
        X = tt_round(qtt_add(qtt_scale(X, 2.0), qtt_scale(XY, -1.0)), eps, rmax)
        out.append(X)
    return out


def tt_svd_reversed(A, eps, rmax=None):
    """Algorithm 1 run from the last mode to the first.

    The right-to-left chain of low-rank approximations: Algorithm 1 applied to
    the tensor with its mode order reversed, with the cores reversed back and
    transposed.  The truncations happen at the same bonds with the same
    tolerance; cores 2..d come out right-orthonormal.
    """
    d = A.ndim
    rev = tt_svd(A.transpose(list(range(d))[::-1]), eps, rmax)
    return [G.transpose(2, 1, 0) for G in rev[::-1]]


def qtt_from_dense_reversed(A, eps, rmax=None):
    cores = tt_svd_reversed(qtt_tensorize(A), eps, rmax)
    return [G.reshape(G.shape[0], 2, 2, G.shape[2]) for G in cores]
