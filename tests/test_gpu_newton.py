"""GPU parity of the Newton-step building blocks and solve against the oracle."""

import numpy as np
import pytest

import scenes
from oracle import pdip, tt
from tests import cases, helpers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_1808_02558_amd import binding
    c = binding.Context()
    yield c
    c.close()


def dev(torch, a, dtype=None):
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def load_matrix(torch, snap, it):
    S = snap["result"].history[it]["S"]
    Spad = helpers.pad_matrix(S, snap["slot"], snap["log2n"])
    rp, col, val = helpers.to_bsr3(Spad, snap["log2n"])
    return Spad, dev(torch, rp), dev(torch, col), dev(torch, val)


@pytest.mark.parametrize("name", ["small_box", "lattice_box"])
def test_bsr_spmv_matches_scipy(torch, ctx, name):
    snap = cases.newton_snapshots(name)
    d = snap["log2n"]
    Spad, rp, col, val = load_matrix(torch, snap, 0)
    x = scenes.tensors.random_vector(1 << d, seed=11)
    y = torch.empty(1 << d, dtype=torch.float64, device="cuda")
    ctx.qtp_bsr_spmv(d, rp, col, val, dev(torch, x), y)
    ref = Spad @ x
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-14, err


@pytest.mark.parametrize("d,rmax,seed", [(6, 8, 1), (10, 16, 2), (14, 24, 3),
                                         (16, 64, 4)])
def test_qtt_apply_f64(torch, ctx, d, rmax, seed):
    ranks = scenes.tensors.random_ranks(d, rmax, seed)
    cores = scenes.tensors.random_qtt_cores(ranks, seed)
    x = scenes.tensors.random_vector(1 << d, seed + 100)
    ref = tt.qtt_matvec(cores, x)
    if d <= 10:
        ref_dense = tt.qtt_to_dense(cores) @ x
        assert np.abs(ref - ref_dense).max() <= 1e-12 * np.abs(ref_dense).max()
    y = torch.empty(1 << d, dtype=torch.float64, device="cuda")
    ctx.qtp_qtt_apply(d, ranks, dev(torch, helpers.flat_cores(cores)), "f64",
                      dev(torch, x), y)
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err


@pytest.mark.parametrize("prec,tol", [("f32", 2e-5), ("bf16", 3e-2)])
def test_qtt_apply_reduced_precision(torch, ctx, prec, tol):
    d, rmax, seed = 12, 32, 7
    ranks = scenes.tensors.random_ranks(d, rmax, seed)
    cores = scenes.tensors.random_qtt_cores(ranks, seed)
    x = scenes.tensors.random_vector(1 << d, seed + 100)
    ref = tt.qtt_matvec(cores, x)
    flat = helpers.flat_cores(cores)
    if prec == "f32":
        c = dev(torch, flat.astype(np.float32))
    else:
        c = dev(torch, flat, torch.float32).to(torch.bfloat16).view(torch.int16)
    y = torch.empty(1 << d, dtype=torch.float64, device="cuda")
    ctx.qtp_qtt_apply(d, ranks, c, prec, dev(torch, x), y)
    err = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < tol, err


@pytest.mark.parametrize("name,it", [("small_box", 0), ("small_box", 5),
                                     ("lattice_box", 0), ("lattice_box", 3)])
def test_newton_solve_block_jacobi_fgmres(torch, ctx, name, it):
    """FGMRES with the block-Jacobi part of the preconditioner only (X = I)."""
    snap = cases.newton_snapshots(name)
    d = snap["log2n"]
    Spad, rp, col, val = load_matrix(torch, snap, it)
    rhs = helpers.pad_vector(snap["result"].history[it]["rhs"], snap["slot"], d)
    xref = helpers.pad_vector(snap["result"].history[it]["dgamma"], snap["slot"], d)
    ctx.qtp_set_config(solve_mode=1, solve_tol=1e-12, fgmres_restart=30,
                       fgmres_maxit=3000)
    ctx.qtp_set_newton_matrix(d, rp, col, val)
    # identity QTT as X: rank-1 cores
    ident = helpers.flat_cores(tt.qtt_identity(d))
    ctx.qtp_precond_load_qtt(d, [1] * (d + 1), dev(torch, ident))
    x = torch.empty(1 << d, dtype=torch.float64, device="cuda")
    rc, st = ctx.qtp_newton_solve(dev(torch, rhs), x)
    xs = x.cpu().numpy()
    res = np.linalg.norm(rhs - Spad @ xs) / np.linalg.norm(rhs)
    assert rc == 0 and res <= 1.01e-12, (rc, res, st.iterations)
    fwd = np.linalg.norm(xs - xref) / np.linalg.norm(xref)
    assert fwd <= 1e-8, fwd


@pytest.mark.parametrize("restart", [1, 5, 32])
def test_fgmres_restart_cycles_match_oracle(torch, ctx, restart):
    """Restart cycles and the lagged convergence test: the GPU solve stops at
    the oracle's iteration count (within rounding) and meets the residual."""
    from oracle import krylov, precond
    snap = cases.newton_snapshots("small_box")
    d = snap["log2n"]
    it = 5
    Spad, rp, col, val = load_matrix(torch, snap, it)
    rhs = helpers.pad_vector(snap["result"].history[it]["rhs"], snap["slot"], d)
    Linv = precond.block_jacobi_inverse_factors(Spad.toarray())
    _, its_ref, _ = krylov.fgmres(lambda v: Spad @ v, lambda v: Linv.T @ (Linv @ v),
                                  rhs, tol=1e-10, restart=restart, maxit=5000)
    ctx.qtp_set_config(solve_mode=1, solve_tol=1e-10, fgmres_restart=restart,
                       fgmres_maxit=5000)
    ctx.qtp_set_newton_matrix(d, rp, col, val)
    ident = helpers.flat_cores(tt.qtt_identity(d))
    ctx.qtp_precond_load_qtt(d, [1] * (d + 1), dev(torch, ident))
    x = torch.empty(1 << d, dtype=torch.float64, device="cuda")
    rc, st = ctx.qtp_newton_solve(dev(torch, rhs), x)
    res = np.linalg.norm(rhs - Spad @ x.cpu().numpy()) / np.linalg.norm(rhs)
    assert rc == 0 and res <= 1.01e-10, (rc, res, st.iterations)
    assert abs(st.iterations - its_ref) <= max(2, its_ref // 20), (st.iterations, its_ref)


def test_newton_solve_with_oracle_qtt_inverse(torch, ctx):
    """Direct solve with a QTT inverse plus refinement (tiny box, 2^9)."""
    snap = cases.newton_snapshots("tiny_box")
    d = snap["log2n"]
    it = 2
    Spad, rp, col, val = load_matrix(torch, snap, it)
    # oracle: block-Jacobi scaled matrix, its dense inverse, QTT by Algorithm 1
    A = Spad.toarray()
    n = A.shape[0]
    L = np.eye(n)
    for s in range(n // 3):
        b = slice(3 * s, 3 * s + 3)
        L[b, b] = np.linalg.cholesky(A[b, b])
    Li = np.linalg.inv(L)
    Xd = np.linalg.inv(Li @ A @ Li.T)
    cores = tt.qtt_from_dense(Xd, 1e-10)
    ranks = helpers.qtt_ranks(cores)
    rhs = helpers.pad_vector(snap["result"].history[it]["rhs"], snap["slot"], d)
    ctx.qtp_set_config(solve_mode=0, solve_tol=1e-10, fgmres_maxit=50)
    ctx.qtp_set_newton_matrix(d, rp, col, val)
    ctx.qtp_precond_load_qtt(d, ranks, dev(torch, helpers.flat_cores(cores)))
    x = torch.empty(1 << d, dtype=torch.float64, device="cuda")
    rc, st = ctx.qtp_newton_solve(dev(torch, rhs), x)
    xs = x.cpu().numpy()
    res = np.linalg.norm(rhs - Spad @ xs) / np.linalg.norm(rhs)
    assert rc == 0 and res <= 1e-10, (rc, res, st.iterations)
    assert st.iterations <= 5
