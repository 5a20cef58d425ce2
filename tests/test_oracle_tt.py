"""Pins of the oracle's TT/QTT toolkit against closed forms and brute force."""

import numpy as np
import pytest

import scenes
from oracle import tt


def test_sine_example_ranks_and_storage():
    # Sec. 3.1 worked example: sin(x+y+z) on n^3 points has TT ranks (2, 2)
    # and 2n + 4n + 2n = 8n stored numbers.
    n = 16
    x = np.linspace(0.0, 1.0, n)
    A = np.sin(x[:, None, None] + x[None, :, None] + x[None, None, :])
    cores = tt.tt_svd(A, 1e-12)
    assert tt.tt_ranks(cores) == [2, 2]
    assert sum(G.size for G in cores) == 8 * n
    assert np.abs(tt.tt_full(cores) - A).max() < 1e-13


@pytest.mark.parametrize("d", [4, 6, 8, 10])
def test_laplacian_qtt_ranks_are_three(d):
    # 1-D Dirichlet Laplacian tridiag(-1, 2, -1): QTT ranks exactly 3
    N = 1 << d
    L = 2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
    q = tt.qtt_from_dense(L, 1e-12)
    assert helpers_ranks(q) == [3] * (d - 1)
    assert np.abs(tt.qtt_to_dense(q) - L).max() < 1e-12


def helpers_ranks(q):
    return [int(G.shape[3]) for G in q[:-1]]


@pytest.mark.parametrize("d", [6, 8])
def test_laplacian_inverse_ranks_at_most_five(d):
    # The inverse (a rank-one-modified min(i,j) kernel) has QTT ranks
    # 4, 5, ..., 5, 4: each level's blocks span at most 5 dimensions.
    N = 1 << d
    L = 2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
    q = tt.qtt_from_dense(np.linalg.inv(L), 1e-12)
    assert helpers_ranks(q) == [4] + [5] * (d - 3) + [4]


def test_identity_ranks_one():
    q = tt.qtt_from_dense(np.eye(256), 1e-12)
    assert helpers_ranks(q) == [1] * 7


def test_random_tt_round_trip_recovers_ranks():
    ranks = [1, 3, 5, 4, 2, 1]
    cores = [c.reshape(c.shape[0], 4, c.shape[3])
             for c in scenes.tensors.random_qtt_cores(ranks, seed=3)]
    A = tt.tt_full(cores)
    rec = tt.tt_svd(A, 1e-12)
    assert tt.tt_ranks(rec) == ranks[1:-1]
    assert np.abs(tt.tt_full(rec) - A).max() < 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("eps", [0.05, 0.2, 0.5])
def test_truncation_error_bound(eps):
    A = np.random.default_rng(5).standard_normal((64, 64))
    q = tt.qtt_from_dense(A, eps)
    err = np.linalg.norm(tt.qtt_to_dense(q) - A) / np.linalg.norm(A)
    assert err <= eps * (1 + 1e-12)
    q2 = tt.qtt_from_dense_reversed(A, eps)
    err2 = np.linalg.norm(tt.qtt_to_dense(q2) - A) / np.linalg.norm(A)
    assert err2 <= eps * (1 + 1e-12)


def test_qtt_matvec_and_entries_on_nonsymmetric_matrix():
    # a transposed (i, j) convention or a reversed bit order fails here
    rng = np.random.default_rng(9)
    A = rng.standard_normal((128, 128))
    q = tt.qtt_from_dense(A, 1e-13)
    x = rng.standard_normal(128)
    assert np.abs(tt.qtt_matvec(q, x) - A @ x).max() < 1e-10
    for (i, j) in [(0, 127), (127, 0), (5, 77), (64, 3)]:
        assert abs(tt.qtt_entry(q, i, j) - A[i, j]) < 1e-11
    # tensorisation: mode k of the tensor is (i_k, j_k), MSB first
    T = tt.qtt_tensorize(A)
    i, j = 0b1010011, 0b0110101
    b = [2 * ((i >> (6 - k)) & 1) + ((j >> (6 - k)) & 1) for k in range(7)]
    assert T[tuple(b)] == A[i, j]


def test_qtt_matmul_and_add():
    rng = np.random.default_rng(2)
    A, B = rng.standard_normal((64, 64)), rng.standard_normal((64, 64))
    qa, qb = tt.qtt_from_dense(A, 1e-13), tt.qtt_from_dense(B, 1e-13)
    assert np.abs(tt.qtt_to_dense(tt.qtt_matmul(qa, qb)) - A @ B).max() < 1e-9
    assert np.abs(tt.qtt_to_dense(tt.qtt_add(qa, qb)) - (A + B)).max() < 1e-11


def test_rounding_removes_redundant_rank():
    N = 256
    L = 2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
    q = tt.qtt_from_dense(L, 1e-12)
    dbl = tt.qtt_add(q, q)
    assert helpers_ranks(dbl) == [6] * 7
    r = tt.tt_round(dbl, 1e-12)
    assert helpers_ranks(r) == [3] * 7
    assert np.abs(tt.qtt_to_dense(r) - 2 * L).max() < 1e-12


def test_rounding_error_bound_and_cap():
    A = np.random.default_rng(4).standard_normal((64, 64))
    q = tt.qtt_from_dense(A, 1e-13)
    for eps in (0.1, 0.3):
        r = tt.tt_round(q, eps)
        err = np.linalg.norm(tt.qtt_to_dense(r) - A) / np.linalg.norm(A)
        assert err <= eps * (1 + 1e-10)
    r = tt.tt_round(q, 1e-13, rmax=3)
    assert max(helpers_ranks(r)) <= 3


def test_newton_schulz_converges_to_inverse():
    d = 6
    N = 1 << d
    L = 2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
    q = tt.qtt_from_dense(L, 1e-12)
    X0 = tt.qtt_scale(tt.qtt_identity(d), 0.25)  # 1/lambda_max bound
    its = tt.newton_schulz(q, X0, 1e-12, 64, 20)
    Li = np.linalg.inv(L)
    errs = [np.linalg.norm(tt.qtt_to_dense(X) - Li) / np.linalg.norm(Li) for X in its]
    assert errs[-1] < 1e-9
    # quadratic phase: the error roughly squares once it is below 1
    k = next(i for i, e in enumerate(errs) if e < 0.1)
    assert errs[k + 1] < 10 * errs[k] ** 2 + 1e-12


def test_reversed_tt_svd_matches_forward_when_exact():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((32, 32))
    f = tt.qtt_from_dense(A, 1e-13)
    r = tt.qtt_from_dense_reversed(A, 1e-13)
    assert helpers_ranks(f) == helpers_ranks(r)
    assert np.abs(tt.qtt_to_dense(r) - A).max() < 1e-12
    # cores 2..d are right-orthonormal
    for G in r[1:]:
        M = G.reshape(G.shape[0], -1)
        assert np.abs(M @ M.T - np.eye(G.shape[0])).max() < 1e-12
