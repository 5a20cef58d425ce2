"""Seeded sphere scenes.

Every scene is a set of spheres (centre, velocity, angular velocity, radius,
mass) inside static container planes, plus the time-step parameters of one
frictional-contact time step (friction coefficient, step size, contact
threshold, gravity) and the exponent d of the padded unknown count 2^d.

The large scenes are *column packings*: spheres are stacked in vertical columns
on a jittered square lattice; the lowest sphere of a column rests exactly on
the highest supporting plane below it and every other sphere rests exactly on
the sphere below it (the height follows from the touching condition).  Lateral
neighbours never overlap (the lattice pitch exceeds the largest diameter plus
the jitter), so they become contacts only through the contact threshold.  This
gives settled, load-carrying contact networks with 2-3 contacts per sphere and
static walls, the structure of the paper's sedimented packings (Section 4),
whose own Chrono scenes are not available.

Masses are part of the input: m = rho * 4/3 * pi * r^3 with rho = 2500 kg/m^3.
Planes are rows (n_x, n_y, n_z, o): unit normal n pointing into the domain and
offset o, so that a point p is inside when n.p - o >= 0.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

RHO = 2500.0
G = 9.81


@dataclasses.dataclass
class Scene:
    name: str
    x: np.ndarray        # [M][3] centres (m)
    v: np.ndarray        # [M][3] velocities (m/s)
    w: np.ndarray        # [M][3] angular velocities (rad/s)
    radius: np.ndarray   # [M]
    mass: np.ndarray     # [M]
    planes: np.ndarray   # [nw][4]
    mu: float
    h: float
    delta: float         # active-set threshold on the gap function
    log2n: int           # padded unknown count is 2**log2n
    gravity: np.ndarray = dataclasses.field(
        default_factory=lambda: np.array([0.0, 0.0, -G]))
    seed: int = 0

    @property
    def M(self) -> int:
        return int(self.x.shape[0])

    @property
    def nw(self) -> int:
        return int(self.planes.shape[0])

    def copy(self) -> "Scene":
        return dataclasses.replace(
            self, x=self.x.copy(), v=self.v.copy(), w=self.w.copy(),
            radius=self.radius.copy(), mass=self.mass.copy(),
            planes=self.planes.copy(), gravity=self.gravity.copy())


def _mass(r):
    return RHO * (4.0 / 3.0) * math.pi * np.asarray(r, dtype=np.float64) ** 3


def _single(name, x, r, planes, mu, h, log2n=3, delta=None):
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    r = np.asarray(r, dtype=np.float64).reshape(-1)
    M = x.shape[0]
    return Scene(name=name, x=x, v=np.zeros((M, 3)), w=np.zeros((M, 3)),
                 radius=r, mass=_mass(r),
                 planes=np.asarray(planes, dtype=np.float64).reshape(-1, 4),
                 mu=float(mu), h=float(h),
                 delta=float(0.1 * r.mean() if delta is None else delta),
                 log2n=log2n)


FLOOR = (0.0, 0.0, 1.0, 0.0)


def sphere_on_plane(r=0.01, mu=0.5, h=1e-3):
    """One sphere resting on the floor z = 0."""
    return _single("sphere_on_plane", [0.0, 0.0, r], [r], [FLOOR], mu, h)


def sphere_on_incline(theta, r=0.01, mu=0.5, h=1e-3):
    """One sphere resting on a plane through the origin tilted by theta about y."""
    n = np.array([-math.sin(theta), 0.0, math.cos(theta)])
    return _single("sphere_on_incline", r * n, [r], [(*n, 0.0)], mu, h)


def stacked_pair(r=0.01, mu=0.5, h=1e-3):
    """Two equal spheres, one exactly on top of the other, on the floor."""
    return _single("stacked_pair", [[0, 0, r], [0, 0, 3 * r]], [r, r],
                   [FLOOR], mu, h, log2n=4)


def three_on_floor(r=0.01, mu=0.5, h=1e-3):
    """Three equal touching spheres in a row on the floor: 5 contacts."""
    return _single("three_on_floor", [[0, 0, r], [2 * r, 0, r], [4 * r, 0, r]],
                   [r, r, r], [FLOOR], mu, h, log2n=4)


def sphere_on_double_floor(r=0.01, mu=0.5, h=1e-3):
    """One sphere on two coincident floor planes (a non-unique split)."""
    return _single("sphere_on_double_floor", [0.0, 0.0, r], [r],
                   [FLOOR, FLOOR], mu, h)


def _column_packing(rng, nx, ny, nz, r_lo, r_hi, pitch, jitter, planes,
                    x_min, y_min):
    """Stack nz spheres in each of nx*ny lattice columns (see module doc)."""
    if r_hi > r_lo:
        r = rng.uniform(r_lo, r_hi, size=(nx, ny, nz))
    else:
        r = np.full((nx, ny, nz), float(r_lo))
    jit = rng.uniform(-jitter, jitter, size=(nx, ny, nz, 2))
    cx = x_min + (np.arange(nx) + 0.5) * pitch
    cy = y_min + (np.arange(ny) + 0.5) * pitch
    px = cx[:, None, None] + jit[..., 0]
    py = cy[None, :, None] + jit[..., 1]
    z = np.empty((nx, ny, nz))
    # lowest sphere: touch the highest supporting plane (n_z > 0) below it
    zb = np.full((nx, ny), -np.inf)
    for n0, n1, n2, o in planes:
        if n2 > 1e-12:
            zb = np.maximum(zb, (o + r[:, :, 0] - n0 * px[:, :, 0]
                                 - n1 * py[:, :, 0]) / n2)
    z[:, :, 0] = zb
    for k in range(1, nz):
        dx = px[:, :, k] - px[:, :, k - 1]
        dy = py[:, :, k] - py[:, :, k - 1]
        s = r[:, :, k] + r[:, :, k - 1]
        z[:, :, k] = z[:, :, k - 1] + np.sqrt(s * s - dx * dx - dy * dy)
    x = np.stack([px, py, z], axis=-1).reshape(-1, 3)
    return x, r.reshape(-1)


def _box_planes(x0, x1, y0, y1, side_walls=True):
    p = [FLOOR]
    if side_walls:
        p += [(1.0, 0.0, 0.0, x0), (-1.0, 0.0, 0.0, -x1),
              (0.0, 1.0, 0.0, y0), (0.0, -1.0, 0.0, -y1)]
    return np.array(p, dtype=np.float64)


def _packing_scene(name, seed, nx, ny, nz, r_lo, r_hi, jitter, pitch, planes,
                   x_min, y_min, mu, h, delta, log2n):
    rng = np.random.default_rng(seed)
    x, r = _column_packing(rng, nx, ny, nz, r_lo, r_hi, pitch, jitter,
                           planes, x_min, y_min)
    M = x.shape[0]
    return Scene(name=name, x=x, v=np.zeros((M, 3)), w=np.zeros((M, 3)),
                 radius=r, mass=_mass(r), planes=planes, mu=mu, h=h,
                 delta=delta, log2n=log2n, seed=seed)


def _box_scene(name, seed, nx, ny, nz, r_lo, r_hi, jitter, pitch_gap, mu, h,
               delta, log2n, side_walls=True):
    pitch = 2.0 * r_hi + 2.0 * jitter + pitch_gap
    X, Y = nx * pitch, ny * pitch
    planes = _box_planes(0.0, X, 0.0, Y, side_walls)
    return _packing_scene(name, seed, nx, ny, nz, r_lo, r_hi, jitter, pitch,
                          planes, 0.0, 0.0, mu, h, delta, log2n)


def lattice_box(seed=1):
    """1,000 spheres of radius 1 cm, 10x10x10 columns in an open-top box.

    Lateral jitter +-0.05 r; mu = 0.5; h = 1e-3 s; padded to 2^13.
    """
    r = 0.01
    return _box_scene("lattice_box", seed, 10, 10, 10, r, r, 0.05 * r, 0.0,
                      0.5, 1e-3, 0.12 * r, 13)


def loose_box(seed=2, nx=32, ny=32, nz=16):
    """16,384 spheres, radius uniform in [0.9, 1.1] cm, in a box; padded to 2^17."""
    return _box_scene("loose_box", seed, nx, ny, nz, 0.009, 0.011, 0.0005,
                      0.0, 0.5, 1e-3, 0.0040, 17)


def hopper(seed=3, nx=64, ny=64, nz=32, theta_deg=30.0):
    """131,072 spheres, radius uniform in [0.8, 1.2] cm, in a rectangular hopper.

    Floor z = 0 for |x| <= a, two planes inclined by theta above it for |x| > a,
    and two vertical side walls in y; mu = 0.4; padded to 2^20.
    """
    r_lo, r_hi, jitter = 0.008, 0.012, 0.0005
    pitch = 2.0 * r_hi + 2.0 * jitter
    X, Y = nx * pitch, ny * pitch
    a = X / 6.0
    th = math.radians(theta_deg)
    s, c = math.sin(th), math.cos(th)
    planes = np.array([
        FLOOR,
        (s, 0.0, c, -a * s),          # left slope, rising for x < -a
        (-s, 0.0, c, -a * s),         # right slope, rising for x > a
        (0.0, 1.0, 0.0, 0.0),
        (0.0, -1.0, 0.0, -Y),
    ])
    return _packing_scene("hopper", seed, nx, ny, nz, r_lo, r_hi, jitter,
                          pitch, planes, -X / 2.0, 0.0, 0.4, 1e-3, 0.0065, 20)


def column_collapse(seed=5, nx=64, ny=64, nz=256):
    """1,048,576 spheres, radius in [0.8, 1.2] cm, on a floor with no side walls."""
    return _box_scene("column_collapse", seed, nx, ny, nz, 0.008, 0.012,
                      0.0005, 0.0, 0.5, 5e-4, 0.0065, 23, side_walls=False)


SCENES = {
    "sphere_on_plane": sphere_on_plane,
    "stacked_pair": stacked_pair,
    "three_on_floor": three_on_floor,
    "sphere_on_double_floor": sphere_on_double_floor,
    "lattice_box": lattice_box,
    "loose_box": loose_box,
    "hopper": hopper,
    "column_collapse": column_collapse,
}


def make_scene(name, **kw):
    return SCENES[name](**kw)
