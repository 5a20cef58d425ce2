"""GPU parity of the time step (detection, assembly, PDIP, integration)."""

import math

import numpy as np
import pytest

import scenes
from oracle import assembly, contacts, pdip, mlp
from tests import cases, helpers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_ctx(torch, sc, **kw):
    from paper_1808_02558_amd import binding
    ctx = binding.Context(**kw)
    ctx.qtp_set_bodies(dev(torch, sc.x), dev(torch, sc.v), dev(torch, sc.w),
                       dev(torch, sc.radius), dev(torch, sc.mass))
    ctx.qtp_set_walls(sc.planes)
    ctx.qtp_set_params(sc.mu, sc.h, sc.delta, sc.gravity, sc.log2n)
    return ctx


def scene(name):
    return cases.LOCAL[name]() if name in cases.LOCAL else scenes.make_scene(name)


@pytest.mark.parametrize("name", ["tiny_box", "small_box", "lattice_box",
                                  "loose_box", "hopper"])
def test_contacts_bit_exact(torch, name):
    sc = scene(name)
    ref = contacts.detect(sc)
    ctx = make_ctx(torch, sc)
    try:
        nc = ctx.qtp_detect()
        g = ctx.qtp_get_contacts(nc)
    finally:
        ctx.close()
    print(f"{name}: {nc} contacts")
    assert nc == ref.nc
    assert np.array_equal(g["a"].cpu().numpy(), ref.a)
    assert np.array_equal(g["b"].cpu().numpy(), ref.b)
    assert np.array_equal(g["key"].cpu().numpy().view(np.uint64), ref.key)
    slot, _ = contacts.slot_map(ref.nc, sc.log2n)
    assert np.array_equal(g["slot"].cpu().numpy(), slot)
    assert np.array_equal(g["phi"].cpu().numpy(), ref.phi)
    assert np.array_equal(g["frame"].cpu().numpy().reshape(-1, 3, 3), ref.frame)


@pytest.mark.parametrize("name", ["tiny_box", "lattice_box", "loose_box"])
def test_assembly_matches_oracle(torch, name):
    sc = scene(name)
    c = contacts.detect(sc)
    N, r, D = assembly.qp_data(sc, c)
    gbar, vbar = assembly.scales(sc)
    Ns, rs = (N * (gbar / vbar)).tocsr(), r / vbar
    slot, _ = contacts.slot_map(c.nc, sc.log2n)
    Npad = helpers.pad_matrix(Ns, slot, sc.log2n)
    ctx = make_ctx(torch, sc)
    try:
        ctx.qtp_detect()
        ctx.qtp_assemble()
        rp, col, val, rg = ctx.qtp_get_qp(sc.log2n)
    finally:
        ctx.close()
    rp_o, col_o, val_o = helpers.to_bsr3(Npad, sc.log2n)
    assert np.array_equal(rp.cpu().numpy(), rp_o)
    assert np.array_equal(col.cpu().numpy(), col_o)
    vg = val.cpu().numpy()
    assert np.abs(vg - val_o).max() <= 1e-13 * np.abs(val_o).max()
    rpad = helpers.pad_vector(rs, slot, sc.log2n)
    assert np.abs(rg.cpu().numpy() - rpad).max() <= 1e-12 * np.abs(rpad).max()


@pytest.mark.parametrize("name", ["tiny_box", "small_box", "lattice_box"])
def test_pdip_step_matches_oracle(torch, name):
    sc = scene(name)
    c, res, gamma_o, (x_o, v_o, w_o) = pdip.time_step(sc)
    assert res.converged
    ctx = make_ctx(torch, sc, solve_tol=1e-10, fgmres_maxit=5000, ns_iters=6)
    try:
        ctx.qtp_detect()
        ctx.qtp_assemble()
        rc, st = ctx.qtp_pdip_solve()
        g = ctx.qtp_get_impulses(c.nc).cpu().numpy().reshape(-1)
        Y = ctx.qtp_mlp_targets(c.nc).cpu().numpy().astype(np.float64)
        ctx.qtp_integrate()
        x, v, w = (t.cpu().numpy() for t in ctx.qtp_get_state(sc.M))
    finally:
        ctx.close()
    print(f"{name}: PDIP {st.pdip_iterations} (oracle {res.iterations}) FGMRES "
          f"{st.fgmres_iterations} max {st.max_fgmres} precond {st.ms_precond:.1f} ms "
          f"solve {st.ms_solve:.1f} ms")
    assert rc == 0 and st.converged
    err = np.linalg.norm(g - gamma_o) / np.linalg.norm(gamma_o)
    assert err <= 1e-6, err
    vscale = np.linalg.norm(sc.gravity) * sc.h
    assert np.abs(v - v_o).max() <= 1e-6 * vscale
    assert np.abs(x - x_o).max() <= 1e-6 * vscale * sc.h
    # training targets of the warm start, from the oracle's impulses
    gbar = sc.mass.mean() * np.linalg.norm(sc.gravity) * sc.h
    Yo = mlp.targets(gamma_o / gbar, sc.mu)
    big = gamma_o.reshape(-1, 3)[:, 0] >= 1e-3 * gbar
    assert np.isfinite(Y).all()
    assert np.abs(Y - Yo)[big].max() <= 1e-4


@pytest.mark.parametrize("theta,mu", [(0.0, 0.5), (0.3, 0.5), (math.pi / 6, 0.05)])
def test_closed_forms_through_the_abi(torch, theta, mu):
    sc = scenes.sphere_on_incline(theta, mu=mu) if theta else scenes.sphere_on_plane()
    ctx = make_ctx(torch, sc)
    try:
        rc, st = ctx.qtp_step()
        # qtp_step integrates; impulses of the solve are still readable
        g = ctx.qtp_get_impulses(1).cpu().numpy()[0]
        x, v, w = (t.cpu().numpy() for t in ctx.qtp_get_state(1))
    finally:
        ctx.close()
    mgh = sc.mass[0] * 9.81 * sc.h
    gn, gt = g[0] / mgh, math.hypot(g[1], g[2]) / mgh
    if theta == 0.0:
        assert abs(gn - 1) < 1e-6 and gt < 1e-9 and np.abs(v).max() < 1e-8
    elif math.tan(theta) <= 3.5 * mu:
        assert abs(gn - math.cos(theta)) < 1e-6
        assert abs(gt - 2 / 7 * math.sin(theta)) < 1e-6
    else:
        en = (math.cos(theta) + mu * math.sin(theta)) / (1 + 3.5 * mu * mu)
        assert abs(gn - en) < 1e-6 and abs(gt - mu * en) < 1e-6


@pytest.mark.parametrize("name,shift", [("lattice_box", 0.3), ("loose_box", 0.3),
                                        ("lattice_box", None)])
def test_persistent_slots_match_oracle(torch, name, shift):
    """Two configurations in a row with slot re-use: the second step's slots
    (kept, filled forward, or rebuilt) and its assembled matrix match the
    oracle bit for bit / to rounding."""
    import dataclasses
    sc = scene(name)
    rng = np.random.default_rng(17)
    if shift is None:  # equal radii: permuting the positions renames the bodies
        x2 = sc.x[rng.permutation(sc.M)]
    else:
        x2 = sc.x + rng.uniform(-shift, shift, sc.x.shape) * sc.delta
    sc2 = dataclasses.replace(sc, x=np.ascontiguousarray(x2))
    d = sc.log2n
    c1 = contacts.detect(sc)
    s1, _ = contacts.slot_map(c1.nc, d)
    c2 = contacts.detect(sc2)
    s2, pers, rebuilt = contacts.slot_map_persistent(c1.a, c1.b, s1, c2.a, c2.b, d)
    ctx = make_ctx(torch, sc, slot_mode=1)
    try:
        n1 = ctx.qtp_detect()
        g1 = ctx.qtp_get_contacts(n1)
        ctx.qtp_set_bodies(dev(torch, sc2.x), dev(torch, sc2.v), dev(torch, sc2.w),
                           dev(torch, sc2.radius), dev(torch, sc2.mass))
        n2 = ctx.qtp_detect()
        g2 = ctx.qtp_get_contacts(n2)
        ctx.qtp_assemble()
        rp, col, val, rg = ctx.qtp_get_qp(d)
    finally:
        ctx.close()
    print(f"{name}: {c1.nc} -> {c2.nc} contacts, {int(pers.sum())} kept their slot, "
          f"rebuilt {rebuilt}")
    assert np.array_equal(g1["slot"].cpu().numpy(), s1)
    assert n2 == c2.nc
    assert np.array_equal(g2["a"].cpu().numpy(), c2.a)
    assert np.array_equal(g2["slot"].cpu().numpy(), s2)
    N, r, D = assembly.qp_data(sc2, c2)
    gbar, vbar = assembly.scales(sc2)
    Npad = helpers.pad_matrix((N * (gbar / vbar)).tocsr(), s2, d)
    rp_o, col_o, val_o = helpers.to_bsr3(Npad, d)
    assert np.array_equal(rp.cpu().numpy(), rp_o)
    assert np.array_equal(col.cpu().numpy(), col_o)
    assert np.abs(val.cpu().numpy() - val_o).max() <= 1e-13 * np.abs(val_o).max()
    rpad = helpers.pad_vector(r / vbar, s2, d)
    assert np.abs(rg.cpu().numpy() - rpad).max() <= 1e-12 * np.abs(rpad).max()


def test_previous_step_start(torch):
    """Two time steps with slot re-use; the second starts from the first's
    impulses (warm_start = 1) and reaches the cold start's solution."""
    sc = cases.small_box()
    cfg = dict(solve_tol=1e-10, fgmres_maxit=5000, qtt_mode=0, slot_mode=1)
    out = {}
    for ws in (0, 1):
        ctx = make_ctx(torch, sc, warm_start=ws, **cfg)
        try:
            ctx.qtp_step()
            rc, st = ctx.qtp_step()
            g = ctx.qtp_get_impulses(st.n_contacts).cpu().numpy()
            x, v, w = (t.cpu().numpy() for t in ctx.qtp_get_state(sc.M))
        finally:
            ctx.close()
        out[ws] = (rc, st, g, v)
    (rc0, cold, g0, v0), (rc1, warm, g1, v1) = out[0], out[1]
    print(f"second step: cold {cold.pdip_iterations} PDIP its, previous-step start "
          f"{warm.pdip_iterations} (fallback {warm.warm_fallback}), "
          f"{warm.persistent_contacts} of {warm.n_contacts} contacts kept their slot")
    assert rc0 == 0 and rc1 == 0
    assert warm.warm_started == 1 and warm.persistent_contacts > 0
    assert np.linalg.norm(g1 - g0) <= 1e-4 * np.linalg.norm(g0)
    assert np.abs(v1 - v0).max() <= 1e-6 * np.linalg.norm(sc.gravity) * sc.h
