"""Pins of the oracle's contact model and PDIP against closed forms."""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import scenes
from oracle import assembly, contacts, pdip
from tests import cases

G = 9.81


def step(sc):
    c, res, gamma, state = pdip.time_step(sc)
    assert res.converged
    return c, res, gamma.reshape(-1, 3), state


def test_sphere_on_plane_normal_impulse_is_mgh():
    sc = scenes.sphere_on_plane()
    c, res, g, (x, v, w) = step(sc)
    mgh = sc.mass[0] * G * sc.h
    assert c.nc == 1
    assert abs(g[0, 0] / mgh - 1) < 1e-6 and np.abs(g[0, 1:]).max() < 1e-9 * mgh
    assert np.abs(v).max() < 1e-8 and np.abs(w).max() < 1e-8


@pytest.mark.parametrize("theta,mu", [(0.3, 0.5), (math.pi / 6, 0.05),
                                      (0.2, 0.02), (0.6, 1.0)])
def test_sphere_on_incline(theta, mu):
    # CCP closed forms: rolling if tan(theta) <= 3.5 mu, else sliding with the
    # cone-relaxation lift gamma_n = mgh (cos + mu sin) / (1 + 3.5 mu^2).
    sc = scenes.sphere_on_incline(theta, mu=mu)
    c, res, g, _ = step(sc)
    mgh = sc.mass[0] * G * sc.h
    gn, gt = g[0, 0] / mgh, np.hypot(g[0, 1], g[0, 2]) / mgh
    if math.tan(theta) <= 3.5 * mu:
        assert abs(gn - math.cos(theta)) < 1e-6
        assert abs(gt - 2.0 / 7.0 * math.sin(theta)) < 1e-6
    else:
        en = (math.cos(theta) + mu * math.sin(theta)) / (1 + 3.5 * mu * mu)
        assert abs(gn - en) < 1e-6
        assert abs(gt - mu * en) < 1e-6


def test_stacked_pair_loads():
    sc = scenes.stacked_pair()
    c, res, g, _ = step(sc)
    mgh = sc.mass[0] * G * sc.h
    floor = c.b >= c.M
    assert abs(g[floor][0, 0] / mgh - 2) < 1e-6
    assert abs(g[~floor][0, 0] / mgh - 1) < 1e-6


def test_double_floor_splits_evenly():
    sc = scenes.sphere_on_double_floor()
    c, res, g, (x, v, w) = step(sc)
    mgh = sc.mass[0] * G * sc.h
    assert np.allclose(g[:, 0] / mgh, 0.5, atol=1e-6)
    assert np.abs(v).max() < 1e-8


def test_sphere_on_plane_newton_matrix_entries():
    sc = scenes.sphere_on_plane()
    c = contacts.detect(sc)
    N, r, D = assembly.qp_data(sc, c)
    m = sc.mass[0]
    assert np.allclose(N.toarray(), np.diag([1 / m, 3.5 / m, 3.5 / m]), rtol=1e-14)
    assert abs(r[0] + G * sc.h) < 1e-15  # resting: Phi = 0, v_free = -g h


def test_three_on_floor_block_pattern_is_line_graph():
    # Sec. 3.3: block (i, j) of N is non-zero iff contacts i and j share a body
    sc = scenes.three_on_floor()
    c = contacts.detect(sc)
    N, r, D = assembly.qp_data(sc, c)
    assert c.nc == 5
    bodies = [{int(a), int(b)} - {sc.M + w for w in range(sc.nw)}
              for a, b in zip(c.a, c.b)]
    B = np.abs(N.toarray()).reshape(5, 3, 5, 3).sum(axis=(1, 3)) > 0
    for i in range(5):
        for j in range(5):
            assert B[i, j] == bool(bodies[i] & bodies[j])


def test_newton_matrix_symmetric_psd_and_momentum_balance():
    snap = cases.newton_snapshots("tiny_box")
    N = snap["N"].toarray()
    assert np.abs(N - N.T).max() < 1e-12 * np.abs(N).max()
    assert np.linalg.eigvalsh(N).min() > -1e-10 * np.abs(N).max()
    # P5: sum of contact impulses on bodies equals the momentum change
    sc = snap["scene"]
    c, res, gamma, (x, v, w) = pdip.time_step(sc)
    D = assembly.jacobian(sc, c)
    imp = (D @ gamma).reshape(-1, 2, 3)[:, 0, :].sum(0)
    dp = (sc.mass[:, None] * (v - sc.v)).sum(0) - sc.h * sc.mass.sum() * sc.gravity
    assert np.abs(imp - dp).max() < 1e-12 * sc.mass.sum() * G * sc.h


def test_kkt_and_cone_complementarity():
    snap = cases.newton_snapshots("tiny_box")
    res, N, r, mu = snap["result"], snap["N"], snap["r"], snap["scene"].mu
    g = res.gamma.reshape(-1, 3)
    assert res.converged
    # primal feasibility: inside the friction cone
    assert np.all(np.hypot(g[:, 1], g[:, 2]) <= mu * g[:, 0] * (1 + 1e-12))
    # dual feasibility of the CCP: u_n - mu |u_t| >= -tol (relaxed complementarity)
    u = (N @ res.gamma + r).reshape(-1, 3)
    assert np.all(u[:, 0] - mu * np.hypot(u[:, 1], u[:, 2]) >= -1e-3)
    # complementarity gap per contact bounded by the surrogate gap
    assert np.all(np.abs((g * u).sum(1)) <= 1e-3 + res.gap)
    assert res.gap / (2 * g.shape[0]) <= 1e-8


def test_schur_complement_equals_unreduced_newton_step():
    snap = cases.newton_snapshots("tiny_box")
    h = snap["result"].history[3]
    N, r, mu = snap["N"], snap["r"], snap["scene"].mu
    A, b = pdip.unreduced_system(N, r, h["gamma"], h["lam"], mu, h["t"])
    y = sp.linalg.spsolve(A.tocsc(), b)
    n = h["gamma"].size
    assert np.abs(y[:n] - h["dgamma"]).max() <= 1e-9 * np.abs(h["dgamma"]).max()
    assert np.abs(y[n:] - h["dlam"]).max() <= 1e-9 * np.abs(h["dlam"]).max()


def test_celllist_equals_bruteforce():
    sc = scenes.lattice_box()
    a1, b1 = contacts.sphere_pairs_bruteforce(sc.x, sc.radius, sc.delta)
    a2, b2 = contacts.sphere_pairs_celllist(sc.x, sc.radius, sc.delta)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


def test_contact_order_frames_and_slots():
    sc = scenes.lattice_box()
    c = contacts.detect(sc)
    assert np.all(np.diff(c.key.astype(np.float64)) >= 0)
    F = c.frame
    gram = np.einsum("nij,nkj->nik", F, F)
    assert np.abs(gram - np.eye(3)).max() < 1e-14
    det = np.linalg.det(F)
    assert np.allclose(det, 1.0)
    slot, dummy = contacts.slot_map(c.nc, sc.log2n)
    S = (1 << sc.log2n) // 3
    assert np.all(np.diff(slot) >= 1) and slot[-1] < S
    assert dummy.sum() == S - c.nc
    with pytest.raises(ValueError):
        contacts.slot_map(S + 1, sc.log2n)


def test_slot_map_hierarchy_example():
    # Fig. "hierarchyevolve": 5 pairs in a tree of 8 leaves; dummies fill the rest
    slot, dummy = contacts.slot_map(5, 4)  # 16 unknowns -> 5 slots
    assert list(slot) == [0, 1, 2, 3, 4] and not dummy.any()
    slot, dummy = contacts.slot_map(3, 4)
    assert list(slot) == [0, 1, 3] and list(np.nonzero(dummy)[0]) == [2, 4]


def test_persistent_slots_reduce_to_the_fresh_map():
    """No previous contacts: every contact is new and takes its fresh slot."""
    a = np.arange(7)
    b = a + 100
    slot, pers, rebuilt = contacts.slot_map_persistent([], [], [], a, b, 5)
    fresh, _ = contacts.slot_map(7, 5)
    assert not rebuilt and not pers.any()
    assert np.array_equal(slot, fresh)


def test_persistent_slots_keep_the_tree_and_fill_forward():
    """Hand-worked case on 2^5 (10 slots): contacts (0,1) (2,3) (4,5) sat in
    slots 0, 3, 6; now (2,3) is gone and two new contacts appear around the
    persistent ones."""
    prev_a, prev_b, prev_s = [0, 2, 4], [1, 3, 5], [0, 3, 6]
    a = np.array([0, 7, 4, 8])
    b = np.array([1, 9, 5, 10])
    slot, pers, rebuilt = contacts.slot_map_persistent(prev_a, prev_b, prev_s, a, b, 5)
    # fresh slots floor(q * 10 / 4) = 0, 2, 5, 7; persistent keep 0 and 6;
    # (7,9) takes 2; (8,10) takes the first free slot >= max(7, 3) = 7
    assert not rebuilt
    assert pers.tolist() == [True, False, True, False]
    assert slot.tolist() == [0, 2, 6, 7]


def test_persistent_slots_rebuild_when_no_slot_is_left():
    """The last new contact finds no free slot after its fresh one: rebuild."""
    prev_a, prev_b, prev_s = [0], [1], [9]
    a = np.array([2, 0])
    b = np.array([3, 1])
    # 2^5 -> 10 slots; new (2,3) has fresh slot 0, persistent (0,1) keeps 9
    slot, pers, rebuilt = contacts.slot_map_persistent(prev_a, prev_b, prev_s, a, b, 5)
    assert not rebuilt and slot.tolist() == [0, 9]
    # many new contacts behind a persistent one in the last slot
    a = np.array([0] + list(range(2, 11)))
    b = np.array([1] + list(range(102, 111)))
    slot, pers, rebuilt = contacts.slot_map_persistent(prev_a, prev_b, prev_s, a, b, 5)
    fresh, _ = contacts.slot_map(10, 5)
    assert rebuilt and np.array_equal(slot, fresh) and not pers.any()


def test_persistent_slots_brute_force_properties():
    """Random small cases: the map is injective, persistent contacts keep
    their slots, and new contacts are increasing and at or after their fresh
    slots."""
    rng = np.random.default_rng(11)
    for trial in range(200):
        d = int(rng.integers(4, 8))
        S = (1 << d) // 3
        n0 = int(rng.integers(0, S + 1))
        pool = rng.permutation(3 * S)[: 2 * S]
        prev = pool[:n0]
        prev_slot = np.sort(rng.permutation(S)[:n0])
        keep = prev[rng.random(n0) < 0.7]
        new = pool[n0: n0 + int(rng.integers(0, S - len(keep) + 1))]
        cur = rng.permutation(np.concatenate([keep, new]))[:S]
        a, b = cur // 1000, cur % 1000 + 1000
        pa, pb = prev // 1000, prev % 1000 + 1000
        slot, pers, rebuilt = contacts.slot_map_persistent(pa, pb, prev_slot, a, b, d)
        assert len(set(slot.tolist())) == len(slot)
        if rebuilt:
            continue
        old = {(int(x), int(y)): int(s) for x, y, s in zip(pa, pb, prev_slot)}
        fresh, _ = contacts.slot_map(len(cur), d)
        last = -1
        for q in range(len(cur)):
            key = (int(a[q]), int(b[q]))
            if key in old:
                assert pers[q] and slot[q] == old[key]
            else:
                assert not pers[q] and slot[q] >= fresh[q] and slot[q] > last
                last = slot[q]
