"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only *generates* inputs: sphere scenes (positions, velocities,
radii, masses, container planes) and random test tensors.  It contains none of
the solver's arithmetic (no contact detection, no assembly, no interior-point
or tensor-train algebra), so that the oracle and the HIP library can both read
the same inputs while sharing no code.
"""

from . import tensors  # noqa: F401
from .packings import (  # noqa: F401
    Scene,
    SCENES,
    make_scene,
    sphere_on_plane,
    sphere_on_incline,
    stacked_pair,
    three_on_floor,
    sphere_on_double_floor,
    lattice_box,
    loose_box,
    hopper,
    column_collapse,
)
