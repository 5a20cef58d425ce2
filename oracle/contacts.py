"""Active contact set, contact frames, Morton ordering and the slot map.

Paper passages followed
-----------------------
* Sec. 2.2: gap function Phi_i (positive apart, zero touching, negative
  overlapping), unit normal n and tangents t1, t2 at the contact, and the
  active set A(q, delta) = {i : Phi_i <= delta}.
* Sec. 3.3: contacts are ordered by a spatial octree hierarchy of their
  positions; the matrix is embedded in a uniform tree of 2^L leaves whose
  unused leaves are dummy unknowns with an identity block.

Readings where the paper is silent
----------------------------------
* The active-set predicate is evaluated as |x_b - x_a|^2 <= (r_a + r_b + delta)^2
  (sphere pairs) and Phi <= delta (sphere-wall), in this operation order and
  without fused multiply-adds, so that another implementation can reproduce
  the list bit for bit.
* Normal: from sphere a to sphere b (a < b); for a wall contact, the wall's
  inward normal (from the wall towards the sphere).  t1 = normalise(n x e_k)
  with e_k the axis of smallest |n_k| (lowest k on ties), t2 = n x t1.
* Octree order: a 63-bit Morton key (21 bits per axis, x most significant)
  of the key point -- the centre midpoint for a sphere pair, the sphere's
  touching point x - r n for a wall -- quantised over the bounding box of the
  spheres; ties broken by (a, b).
* Slot map: 3 unknowns per contact (n, t1, t2), S = floor(2^d / 3) slots, the
  contact of Morton rank q takes slot floor(q * S / Nc), so that dummy slots
  are spread through the hierarchy; the remaining unknowns are dummies.
* A wall w is encoded as body index M + w.
"""

from __future__ import annotations

import numpy as np

MORTON_BITS = 21


def _pair_predicate(x, radius, delta, a, b):
    dx = x[b, 0] - x[a, 0]
    dy = x[b, 1] - x[a, 1]
    dz = x[b, 2] - x[a, 2]
    d2 = (dx * dx + dy * dy) + dz * dz
    s = (radius[a] + radius[b]) + delta
    return d2 <= s * s


def _wall_phi(x, radius, plane):
    n0, n1, n2, o = plane
    return (((n0 * x[:, 0] + n1 * x[:, 1]) + n2 * x[:, 2]) - o) - radius


def sphere_pairs_bruteforce(x, radius, delta):
    """All sphere pairs (a < b) in the active set, by checking every pair."""
    M = x.shape[0]
    a, b = np.triu_indices(M, k=1)
    keep = _pair_predicate(x, radius, delta, a, b)
    return a[keep].astype(np.int64), b[keep].astype(np.int64)


def sphere_pairs_celllist(x, radius, delta):
    """Same set as the brute force, through a uniform cell grid.

    Cells have edge >= 2 max(r) + delta, so every active pair lies in the same
    or in adjacent cells; all 27 neighbour cells are scanned and a < b kept.
    """
    M = x.shape[0]
    if M < 2:
        e = np.zeros(0, np.int64)
        return e, e
    cell = 2.0 * float(radius.max()) + float(delta)
    lo = x.min(axis=0)
    c = np.floor((x - lo) / cell).astype(np.int64)
    dims = c.max(axis=0) + 3
    cid = ((c[:, 0] + 1) * dims[1] + (c[:, 1] + 1)) * dims[2] + (c[:, 2] + 1)
    order = np.argsort(cid, kind="stable")
    sorted_cid = cid[order]
    ncell = int(dims[0] * dims[1] * dims[2])
    start = np.searchsorted(sorted_cid, np.arange(ncell), side="left")
    stop = np.searchsorted(sorted_cid, np.arange(ncell), side="right")
    out_a, out_b = [], []
    for ox in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for oz in (-1, 0, 1):
                nid = cid + (ox * dims[1] + oy) * dims[2] + oz
                cnt = stop[nid] - start[nid]
                ii = np.repeat(np.arange(M), cnt)
                base = np.repeat(start[nid], cnt)
                off = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
                jj = order[base + off]
                m = jj > ii
                ii, jj = ii[m], jj[m]
                keep = _pair_predicate(x, radius, delta, ii, jj)
                out_a.append(ii[keep])
                out_b.append(jj[keep])
    a = np.concatenate(out_a)
    b = np.concatenate(out_b)
    o = np.lexsort((b, a))
    return a[o].astype(np.int64), b[o].astype(np.int64)


def wall_contacts(x, radius, planes, delta):
    """(sphere, wall) pairs with Phi <= delta."""
    s_list, w_list = [], []
    for w in range(planes.shape[0]):
        phi = _wall_phi(x, radius, planes[w])
        idx = np.nonzero(phi <= delta)[0]
        s_list.append(idx)
        w_list.append(np.full(idx.shape, w))
    if not s_list:
        e = np.zeros(0, np.int64)
        return e, e
    return (np.concatenate(s_list).astype(np.int64),
            np.concatenate(w_list).astype(np.int64))


def tangent_basis(n):
    """t1 = normalise(n x e_k), k = argmin |n_k| (first on ties); t2 = n x t1."""
    an = np.abs(n)
    k = np.where((an[:, 0] <= an[:, 1]) & (an[:, 0] <= an[:, 2]), 0,
                 np.where(an[:, 1] <= an[:, 2], 1, 2))
    n0, n1, n2 = n[:, 0], n[:, 1], n[:, 2]
    z = np.zeros_like(n0)
    c = np.where((k == 0)[:, None], np.stack([z, n2, -n1], 1),
                 np.where((k == 1)[:, None], np.stack([-n2, z, n0], 1),
                          np.stack([n1, -n0, z], 1)))
    cn = np.sqrt((c[:, 0] * c[:, 0] + c[:, 1] * c[:, 1]) + c[:, 2] * c[:, 2])
    t1 = c / cn[:, None]
    t2 = np.stack([n1 * t1[:, 2] - n2 * t1[:, 1],
                   n2 * t1[:, 0] - n0 * t1[:, 2],
                   n0 * t1[:, 1] - n1 * t1[:, 0]], 1)
    return t1, t2


def _spread_bits(q):
    q = q.astype(np.uint64)
    out = np.zeros_like(q)
    for i in range(MORTON_BITS):
        out |= ((q >> np.uint64(i)) & np.uint64(1)) << np.uint64(3 * i)
    return out


def morton_keys(p, lo, hi):
    """63-bit Morton key of points p over the box [lo, hi], x most significant."""
    scale = float(1 << MORTON_BITS)
    qmax = (1 << MORTON_BITS) - 1
    q = np.floor(((p - lo) / (hi - lo)) * scale)
    q = np.clip(q, 0, qmax).astype(np.int64)
    return ((_spread_bits(q[:, 0]) << np.uint64(2))
            | (_spread_bits(q[:, 1]) << np.uint64(1))
            | _spread_bits(q[:, 2]))


class Contacts:
    """The ordered active set of one time step.

    Arrays are in Morton order: a, b (b >= M means wall b - M), phi, frame
    [Nc][3][3] (rows n, t1, t2), key (uint64).
    """

    def __init__(self, a, b, phi, frame, key, M):
        self.a, self.b, self.phi, self.frame, self.key = a, b, phi, frame, key
        self.M = M

    @property
    def nc(self):
        return int(self.a.shape[0])

    @property
    def is_wall(self):
        return self.b >= self.M


def detect(scene, method="auto"):
    """Active set, gaps, frames and Morton order of one scene (Sec. 2.2, 3.3)."""
    x, radius, delta = scene.x, scene.radius, scene.delta
    M = x.shape[0]
    if method == "brute" or (method == "auto" and M <= 4000):
        pa, pb = sphere_pairs_bruteforce(x, radius, delta)
    else:
        pa, pb = sphere_pairs_celllist(x, radius, delta)
    ws, ww = wall_contacts(x, radius, scene.planes, delta)

    # sphere pairs: n from a to b, Phi = |x_b - x_a| - r_a - r_b
    dvec = x[pb] - x[pa]
    d2 = (dvec[:, 0] * dvec[:, 0] + dvec[:, 1] * dvec[:, 1]) + dvec[:, 2] * dvec[:, 2]
    dist = np.sqrt(d2)
    if np.any(dist == 0.0):
        raise ValueError("coincident sphere centres")
    n_p = dvec / dist[:, None]
    phi_p = (dist - radius[pa]) - radius[pb]
    key_p = (x[pa] + x[pb]) * 0.5

    # walls: n = inward plane normal, Phi = n.x - o - r
    n_w = scene.planes[ww, :3]
    phi_w = np.empty(ws.shape[0])
    for w in range(scene.planes.shape[0]):
        m = ww == w
        phi_w[m] = _wall_phi(x[ws[m]], radius[ws[m]], scene.planes[w])
    key_w = x[ws] - radius[ws][:, None] * n_w

    a = np.concatenate([pa, ws])
    b = np.concatenate([pb, M + ww])
    n = np.concatenate([n_p, n_w])
    phi = np.concatenate([phi_p, phi_w])
    kp = np.concatenate([key_p, key_w])

    lo = (x - radius[:, None]).min(axis=0)
    hi = (x + radius[:, None]).max(axis=0)
    key = morton_keys(kp, lo, hi)
    order = np.lexsort((b, a, key))
    a, b, n, phi, key = a[order], b[order], n[order], phi[order], key[order]
    t1, t2 = tangent_basis(n)
    frame = np.stack([n, t1, t2], axis=1)
    return Contacts(a, b, phi, frame, key, M)


def slot_map_persistent(prev_a, prev_b, prev_slot, a, b, log2n):
    """Slots that keep persistent contacts in place (Sec. 3.3: the contact set
    changes little between time steps, so the tree of the previous step is
    re-used and only the changed leaves move).

    prev_a, prev_b, prev_slot: the contacts of the previous step and their
    slots (any order); a, b: the current contacts in Morton order.  A contact
    is persistent when the same pair (a, b) was a contact before; it keeps
    its slot.  The other contacts, in Morton order, each take the lowest free
    slot that is at or after its slot in the fresh map, floor(q S / Nc), and
    after the slot the previous new contact took.  When a new contact finds no
    such slot the whole map is rebuilt fresh.

    Returns (slot, persistent mask, rebuilt flag).
    """
    S = (1 << log2n) // 3
    nc = len(a)
    if nc > S:
        raise ValueError(f"{nc} contacts exceed the {S} slots of 2^{log2n}")
    fresh, _ = slot_map(nc, log2n)
    old = {(int(x), int(y)): int(s) for x, y, s in zip(prev_a, prev_b, prev_slot)}
    slot = np.full(nc, -1, np.int64)
    persistent = np.zeros(nc, bool)
    taken = np.zeros(S, bool)
    for q in range(nc):
        s_old = old.get((int(a[q]), int(b[q])))
        if s_old is not None:
            slot[q] = s_old
            persistent[q] = True
            taken[s_old] = True
    last = -1
    for q in range(nc):
        if persistent[q]:
            continue
        s = max(int(fresh[q]), last + 1)
        while s < S and taken[s]:
            s += 1
        if s >= S:
            return fresh, np.zeros(nc, bool), True
        slot[q] = s
        last = s
    return slot, persistent, False


def slot_map(nc, log2n):
    """Slot of each contact (in Morton rank order) and the dummy mask.

    Raises ValueError when the contacts do not fit in floor(2^d / 3) slots.
    """
    S = (1 << log2n) // 3
    if nc > S:
        raise ValueError(f"{nc} contacts exceed the {S} slots of 2^{log2n}")
    if nc == 0:
        return np.zeros(0, np.int64), np.ones(S, bool)
    q = np.arange(nc, dtype=np.int64)
    slot = (q * S) // nc
    dummy = np.ones(S, bool)
    dummy[slot] = False
    return slot, dummy
