"""GPU parity of the learned warm start: features, forward, gradients, Adam,
and what the trained network gains over the cold start."""

import numpy as np
import pytest

import scenes
from oracle import contacts, mlp, pdip
from tests import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def flat(params):
    return np.concatenate([p.reshape(-1) for p in params]).astype(np.float32)


def unflat(v):
    out, o = [], 0
    for fin, fout in zip(mlp.LAYERS[:-1], mlp.LAYERS[1:]):
        out.append(v[o:o + fin * fout].reshape(fin, fout))
        o += fin * fout
        out.append(v[o:o + fout])
        o += fout
    return out


def make_ctx(torch, sc, **kw):
    from paper_1808_02558_amd import binding
    ctx = binding.Context(**kw)
    ctx.qtp_set_bodies(dev(torch, sc.x), dev(torch, sc.v), dev(torch, sc.w),
                       dev(torch, sc.radius), dev(torch, sc.mass))
    ctx.qtp_set_walls(sc.planes)
    ctx.qtp_set_params(sc.mu, sc.h, sc.delta, sc.gravity, sc.log2n)
    return ctx


def test_features_match_oracle(torch):
    sc = cases.small_box()
    sc.v = np.random.default_rng(3).normal(0, 0.01, size=sc.v.shape)
    sc.w = np.random.default_rng(4).normal(0, 1.0, size=sc.w.shape)
    ref = mlp.features(sc, contacts.detect(sc))
    ctx = make_ctx(torch, sc)
    try:
        nc = ctx.qtp_detect()
        ctx.qtp_assemble()
        X = ctx.qtp_mlp_features(nc).cpu().numpy()
    finally:
        ctx.close()
    assert np.abs(X - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


def test_forward_gradients_and_adam_match_oracle(torch):
    from paper_1808_02558_amd import binding
    rng = np.random.default_rng(7)
    params = scenes.tensors.mlp_init(mlp.LAYERS, seed=11)
    X = rng.standard_normal((300, 11))
    Y = rng.standard_normal((300, 3))
    ctx = binding.Context()
    try:
        assert ctx.qtp_mlp_param_count() == flat(params).size
        ctx.qtp_mlp_set_params(dev(torch, flat(params)))
        P = ctx.qtp_mlp_forward(dev(torch, X, torch.float32)).cpu().numpy()
        Pref, _ = mlp.forward(params, X)
        assert np.abs(P - Pref).max() <= 1e-5 * np.abs(Pref).max()
        loss, g = ctx.qtp_mlp_loss_grad(dev(torch, X, torch.float32),
                                        dev(torch, Y, torch.float32))
        lref, gref = mlp.loss_and_grad(params, X, Y)
        assert abs(loss - lref) <= 1e-5 * lref
        gv, gr = g.cpu().numpy(), np.concatenate([q.reshape(-1) for q in gref])
        assert np.linalg.norm(gv - gr) <= 1e-4 * np.linalg.norm(gr)
        # three Adam steps
        state = ([np.zeros_like(p) for p in params], [np.zeros_like(p) for p in params], 0)
        for _ in range(3):
            ctx.qtp_mlp_train_step(dev(torch, X, torch.float32),
                                   dev(torch, Y, torch.float32), lr=1e-3)
            _, gref = mlp.loss_and_grad(params, X, Y)
            state = mlp.adam_step(params, gref, state, lr=1e-3)
        pg = ctx.qtp_mlp_get_params().cpu().numpy()
        assert np.abs(pg - np.concatenate([q.reshape(-1) for q in params])).max() <= 1e-5
    finally:
        ctx.close()


def test_normalisation_matches_oracle_moments(torch):
    from paper_1808_02558_amd import binding
    X = np.random.default_rng(9).normal(3.0, 2.0, size=(5000, 11)).astype(np.float32)
    ctx = binding.Context()
    try:
        ctx.qtp_mlp_fit_normalization(dev(torch, X))
        mean, istd = ctx.qtp_mlp_get_normalization()
    finally:
        ctx.close()
    X64 = X.astype(np.float64)
    assert np.allclose(mean, X64.mean(0), rtol=1e-5)
    assert np.allclose(istd, 1.0 / X64.std(0), rtol=1e-4)


def collect(torch, ctx, sc, steps):
    """Features and solved scaled impulses over a few GPU time steps."""
    from paper_1808_02558_amd import binding  # noqa: F401
    Xs, Ys = [], []
    for _ in range(steps):
        nc = ctx.qtp_detect()
        ctx.qtp_assemble()
        Xs.append(ctx.qtp_mlp_features(nc))
        rc, st = ctx.qtp_pdip_solve()
        assert rc == 0
        Ys.append(ctx.qtp_mlp_targets(nc))
        ctx.qtp_integrate()
    return torch.cat(Xs), torch.cat(Ys)


def test_learned_warm_start_gain(torch):
    """Train on GPU-solved steps of small boxes, then start a held-out PDIP
    from the network: the same solution (PDIP analytic centre) is reached in
    fewer PDIP iterations than from the cold start."""
    cfg = dict(solve_tol=1e-10, fgmres_maxit=5000, ns_iters=4, qtt_rmax=16)
    Xs, Ys = [], []
    for seed in (21, 22, 23):
        sc = cases.small_box(seed)
        ctx = make_ctx(torch, sc, **cfg)
        try:
            X, Y = collect(torch, ctx, sc, 3)
        finally:
            ctx.close()
        Xs.append(X)
        Ys.append(Y)
    X = torch.cat(Xs)
    Y = torch.cat(Ys)
    params = flat(scenes.tensors.mlp_init(mlp.LAYERS, seed=1000))
    sc = cases.small_box(31)
    ctx = make_ctx(torch, sc, warm_start=2, warm_t0=100.0, **cfg)
    try:
        ctx.qtp_mlp_set_params(dev(torch, params))
        ctx.qtp_mlp_fit_normalization(X)
        n = X.shape[0]
        perm = torch.from_numpy(np.random.default_rng(0).permutation(n)).cuda()
        first = last = None
        for epoch in range(60):
            for b0 in range(0, n, 512):
                idx = perm[b0:b0 + 512]
                loss = ctx.qtp_mlp_train_step(X[idx].contiguous(), Y[idx].contiguous(),
                                              lr=2e-3)
                first = loss if first is None else first
                last = loss
        assert last < 0.5 * first, (first, last)
        # held-out step: warm vs cold
        nc = ctx.qtp_detect()
        ctx.qtp_assemble()
        rc, warm = ctx.qtp_pdip_solve()
        gw = ctx.qtp_get_impulses(nc).cpu().numpy()
        ctx.qtp_set_config(warm_start=0)
        rc2, cold = ctx.qtp_pdip_solve()
        gc = ctx.qtp_get_impulses(nc).cpu().numpy()
    finally:
        ctx.close()
    print(f"held-out step: warm {warm.pdip_iterations} PDIP its (fallback "
          f"{warm.warm_fallback}), cold {cold.pdip_iterations}; loss {first:.3f} -> "
          f"{last:.3f}")
    assert rc == 0 and rc2 == 0
    assert warm.warm_started == 2 and not warm.warm_fallback
    # the gain: fewer PDIP iterations than the cold start on the held-out step
    assert warm.pdip_iterations < cold.pdip_iterations
    # both runs converge to the unique velocities; impulses agree to the PDIP
    # tolerance (the analytic centre of the same barrier)
    assert np.linalg.norm(gw - gc) <= 1e-4 * np.linalg.norm(gc)
