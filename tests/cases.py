"""Seeded parity cases built by the oracle (cached per process)."""

from __future__ import annotations

import functools

import numpy as np

import scenes
from oracle import assembly, contacts, pdip


def small_box(seed=1):
    """216 spheres, 6x6x6 columns in a box, padded to 2^11."""
    return scenes.packings._box_scene("small_box", seed, 6, 6, 6, 0.01, 0.01,
                                      0.0005, 0.0, 0.5, 1e-3, 0.0012, 11)


def tiny_box(seed=4):
    """36 spheres, 3x3x4 columns in a box, padded to 2^9."""
    return scenes.packings._box_scene("tiny_box", seed, 3, 3, 4, 0.01, 0.01,
                                      0.0005, 0.0, 0.5, 1e-3, 0.0012, 9)


LOCAL = {"small_box": small_box, "tiny_box": tiny_box}


@functools.lru_cache(maxsize=None)
def newton_snapshots(name):
    """PDIP run of the oracle with the Newton systems of every iteration."""
    sc = LOCAL[name]() if name in LOCAL else scenes.make_scene(name)
    c = contacts.detect(sc)
    N, r, D = assembly.qp_data(sc, c)
    gbar, vbar = assembly.scales(sc)
    Ns = (N * (gbar / vbar)).tocsr()
    rs = r / vbar
    res = pdip.pdip(Ns, rs, sc.mu, record=True)
    slot, dummy = contacts.slot_map(c.nc, sc.log2n)
    return dict(scene=sc, contacts=c, N=Ns, r=rs, result=res, slot=slot,
                log2n=sc.log2n)
