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
