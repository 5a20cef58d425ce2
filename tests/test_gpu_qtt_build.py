"""GPU parity of the QTT preconditioner construction against the oracle."""

import numpy as np
import pytest

from oracle import precond, tt
from tests import cases, helpers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def load(torch, ctx, name, it):
    snap = cases.newton_snapshots(name)
    d = snap["log2n"]
    S = snap["result"].history[it]["S"]
    Spad = helpers.pad_matrix(S, snap["slot"], d)
    rp, col, val = helpers.to_bsr3(Spad, d)
    ctx.qtp_set_newton_matrix(d, dev(torch, rp), dev(torch, col), dev(torch, val))
    return snap, Spad, d


def cores_of(ctx, which):
    ranks, flat = ctx.qtp_get_qtt_cores(which)
    flat = flat.cpu().numpy()
    cores, o = [], 0
    for k in range(len(ranks) - 1):
        sz = ranks[k] * 4 * ranks[k + 1]
        cores.append(flat[o:o + sz].reshape(ranks[k], 2, 2, ranks[k + 1]))
        o += sz
    return ranks, cores


@pytest.mark.parametrize("eps,rmax_s", [(1e-3, 64), (1e-2, 8), (3e-2, 64), (0.3, 64)])
def test_compression_matches_reversed_algorithm1(torch, eps, rmax_s):
    from paper_1808_02558_amd import binding
    ctx = binding.Context(qtt_eps=eps, qtt_rmax_s=rmax_s, ns_iters=0)
    try:
        snap, Spad, d = load(torch, ctx, "tiny_box", 2)
        ctx.qtp_precond_build(0)
        ranks, cores = cores_of(ctx, 0)
    finally:
        ctx.close()
    St, _ = precond.scaled_matrix(Spad.toarray())
    ref = tt.qtt_from_dense_reversed(St, eps, rmax_s)
    assert ranks == helpers.qtt_ranks(ref)
    A_gpu, A_ref = tt.qtt_to_dense(cores), tt.qtt_to_dense(ref)
    nrm = np.linalg.norm(St)
    assert np.linalg.norm(A_gpu - A_ref) <= 1e-9 * nrm
    if max(ranks) < rmax_s:  # truncated by eps alone: Algorithm 1's bound holds
        assert np.linalg.norm(A_gpu - St) <= eps * nrm * (1 + 1e-9)


def test_newton_schulz_inverse_matches_oracle(torch):
    from paper_1808_02558_amd import binding
    eps, rs, rx, iters = 1e-3, 16, 32, 6
    ctx = binding.Context(qtt_eps=eps, qtt_rmax_s=rs, qtt_rmax=rx, ns_iters=iters)
    try:
        snap, Spad, d = load(torch, ctx, "tiny_box", 2)
        ctx.qtp_precond_build(0)
        st = ctx.qtp_get_precond_stats()
        ranks, cores = cores_of(ctx, 1)
    finally:
        ctx.close()
    St, _ = precond.scaled_matrix(Spad.toarray())
    A, X, done, best = precond.build_inverse(St, eps, rs, rx, iters)
    assert st.ns_iterations == done
    assert abs(st.probe_residual - best) <= 1e-8 * max(best, 1e-3)
    Xg, Xo = tt.qtt_to_dense(cores), tt.qtt_to_dense(X)
    assert np.linalg.norm(Xg - Xo) <= 1e-7 * np.linalg.norm(Xo)


@pytest.mark.parametrize("name,it", [("small_box", 3), ("lattice_box", 5)])
def test_fgmres_with_gpu_built_preconditioner(torch, name, it):
    from paper_1808_02558_amd import binding
    ctx = binding.Context(qtt_eps=1e-2, qtt_rmax_s=16, qtt_rmax=32, ns_iters=6,
                          solve_mode=1, solve_tol=1e-12, fgmres_maxit=3000)
    try:
        snap, Spad, d = load(torch, ctx, name, it)
        ctx.qtp_precond_build(0)
        st = ctx.qtp_get_precond_stats()
        rhs = helpers.pad_vector(snap["result"].history[it]["rhs"], snap["slot"], d)
        xref = helpers.pad_vector(snap["result"].history[it]["dgamma"], snap["slot"], d)
        x = torch.empty(1 << d, dtype=torch.float64, device="cuda")
        rc, sst = ctx.qtp_newton_solve(dev(torch, rhs), x)
    finally:
        ctx.close()
    xs = x.cpu().numpy()
    res = np.linalg.norm(rhs - Spad @ xs) / np.linalg.norm(rhs)
    fwd = np.linalg.norm(xs - xref) / np.linalg.norm(xref)
    print(f"{name} it{it}: NS {st.ns_iterations} probe {st.probe_residual:.3e} "
          f"ranks S~ {st.max_rank_s} X {st.max_rank_x} build {st.ms:.1f} ms; "
          f"FGMRES {sst.iterations} it {sst.ms:.2f} ms")
    assert rc == 0 and res <= 1.01e-12 and fwd <= 1e-8, (rc, res, fwd)
