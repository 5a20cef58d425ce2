"""Contact Jacobian, QP data and the semi-implicit update.

Paper passages followed
-----------------------
* Sec. 2.1: each body has 6 velocity unknowns (translation v, rotation w);
  the mass matrix M is diagonal (m I_3 and the inertia per body).
* Sec. 2.2: D_i = [D_n D_1 D_2] maps the three impulses of contact i to the
  forces and torques on the two bodies; the semi-implicit first-order step
  M (v^{k+1} - v^k) = h f + D gamma, q^{k+1} = q^k + h v^{k+1}.
* Sec. 2.3: N = D^T M^-1 D, r = b + D^T M^-1 k, b_i = [Phi_i / h, 0, 0],
  k = M v^k + h f.

Readings
--------
* Spheres: inertia (2/5) m r^2; orientation never enters sphere contact, so
  the velocity unknowns are (v, w) per sphere and no quaternion is integrated.
* Contact point on sphere b (the body the normal points to) is x_b - r_b n,
  on sphere a it is x_a + r_a n.  Impulse gamma_c along c in {n, t1, t2} acts
  on b as +gamma_c c and on a as -gamma_c c, applied at those points, so the
  6x3 block of D for b is [c ; -r_b (n x c)] and for a is [-c ; -r_a (n x c)].
  D^T v is then the velocity of b's contact point relative to a's, expressed
  in (n, t1, t2).
* Walls are static (infinite mass): a wall contact has only the sphere's
  block, with the sphere in the role of b.
* The only body force is gravity.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def inertia(scene):
    return 0.4 * scene.mass * scene.radius ** 2


def cross(u, v):
    return np.stack([u[:, 1] * v[:, 2] - u[:, 2] * v[:, 1],
                     u[:, 2] * v[:, 0] - u[:, 0] * v[:, 2],
                     u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0]], axis=1)


def jacobian(scene, contacts):
    """D in R^{6M x 3Nc} (Sec. 2.2), velocity order (v_b, w_b) per body."""
    M, nc = scene.M, contacts.nc
    rows, cols, vals = [], [], []
    n = contacts.frame[:, 0, :]
    for c in range(3):
        dirc = contacts.frame[:, c, :]
        nxc = cross(n, dirc)
        col = 3 * np.arange(nc) + c
        # body b (sphere pairs) / the sphere (wall contacts)
        wall = contacts.is_wall
        sb = np.where(wall, contacts.a, contacts.b)
        rb = scene.radius[sb]
        for k in range(3):
            rows.append(6 * sb + k)
            cols.append(col)
            vals.append(dirc[:, k])
            rows.append(6 * sb + 3 + k)
            cols.append(col)
            vals.append(-rb * nxc[:, k])
        # body a of sphere pairs
        pa = np.nonzero(~wall)[0]
        sa = contacts.a[pa]
        ra = scene.radius[sa]
        for k in range(3):
            rows.append(6 * sa + k)
            cols.append(col[pa])
            vals.append(-dirc[pa, k])
            rows.append(6 * sa + 3 + k)
            cols.append(col[pa])
            vals.append(-ra * nxc[pa, k])
    D = sp.coo_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(6 * M, 3 * nc)).tocsr()
    return D


def minv_diag(scene):
    """Diagonal of M^-1 in the (v, w) per-body order."""
    I = inertia(scene)
    m = np.repeat(1.0 / scene.mass, 3)
    i = np.repeat(1.0 / I, 3)
    return np.stack([m.reshape(-1, 3), i.reshape(-1, 3)], axis=1).reshape(-1)


def generalized_velocity(scene):
    return np.concatenate([scene.v, scene.w], axis=1).reshape(-1)


def free_velocity(scene):
    """v^k + h M^-1 f with gravity as the only force."""
    v = scene.v + scene.h * scene.gravity[None, :]
    return np.concatenate([v, scene.w], axis=1).reshape(-1)


def qp_data(scene, contacts):
    """N = D^T M^-1 D and r = b + D^T M^-1 k (Sec. 2.3), physical units."""
    D = jacobian(scene, contacts)
    Minv = sp.diags(minv_diag(scene))
    N = (D.T @ Minv @ D).tocsr()
    N.sum_duplicates()
    b = np.zeros(3 * contacts.nc)
    b[0::3] = contacts.phi / scene.h
    # D^T M^-1 k with k = M v + h f is D^T (v + h M^-1 f)
    r = b + D.T @ free_velocity(scene)
    return N, r, D


def scales(scene):
    """Impulse scale m_bar g h and velocity scale g h (scaled units)."""
    g = float(np.linalg.norm(scene.gravity))
    vbar = g * scene.h
    return float(scene.mass.mean()) * vbar, vbar


def integrate(scene, D, gamma):
    """One semi-implicit step (Sec. 2.2): returns new x, v, w."""
    vnew = free_velocity(scene) + minv_diag(scene) * (D @ gamma)
    vw = vnew.reshape(-1, 2, 3)
    v, w = vw[:, 0, :].copy(), vw[:, 1, :].copy()
    x = scene.x + scene.h * v
    return x, v, w
