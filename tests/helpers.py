"""Test-side marshalling between the oracle's SciPy matrices and the library's
BSR3 slot layout (format conversion only)."""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def unknown_index(slot):
    """Padded unknown index 3*slot + c of every contact unknown (contact order)."""
    return (3 * np.asarray(slot)[:, None] + np.arange(3)[None, :]).ravel()


def pad_matrix(S, slot, log2n):
    """Embed a 3Nc x 3Nc matrix into the 2^d padded layout (identity dummies)."""
    n = 1 << log2n
    idx = unknown_index(slot)
    S = sp.csr_matrix(S)
    coo = S.tocoo()
    rows = idx[coo.row]
    cols = idx[coo.col]
    mask = np.ones(n, bool)
    mask[idx] = False
    dummy = np.nonzero(mask)[0]
    r = np.concatenate([rows, dummy])
    c = np.concatenate([cols, dummy])
    v = np.concatenate([coo.data, np.ones(dummy.size)])
    return sp.csr_matrix((v, (r, c)), shape=(n, n))


def pad_vector(x, slot, log2n):
    out = np.zeros(1 << log2n)
    out[unknown_index(slot)] = x
    return out


def to_bsr3(Spad, log2n):
    """Padded CSR -> (row_ptr, col, val) BSR3 arrays over floor(n/3) slots."""
    n = 1 << log2n
    S = n // 3
    A = sp.csr_matrix(Spad[:3 * S, :3 * S])
    B = sp.bsr_matrix(A, blocksize=(3, 3))
    B.sort_indices()
    # make sure every slot has its diagonal block (dummies: identity)
    return (B.indptr.astype(np.int32), B.indices.astype(np.int32),
            np.ascontiguousarray(B.data.reshape(-1)).astype(np.float64))


def flat_cores(cores):
    return np.concatenate([np.ascontiguousarray(G).ravel() for G in cores])


def qtt_ranks(cores):
    return [1] + [int(G.shape[3]) for G in cores]
