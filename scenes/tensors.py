"""Seeded random tensors and vectors (inputs only, no solver arithmetic)."""

from __future__ import annotations

import numpy as np


def random_ranks(d, rmax, seed):
    """Ranks r_0..r_d with r_0 = r_d = 1 and 1 <= r_k <= min(rmax, 4^k, 4^(d-k))."""
    rng = np.random.default_rng(seed)
    r = [1]
    for k in range(1, d):
        cap = min(rmax, 4 ** min(k, d - k))
        r.append(int(rng.integers(max(1, cap // 2), cap + 1)))
    r.append(1)
    return r


def random_qtt_cores(ranks, seed, scale=None):
    """List of cores [r_{k-1}, 2, 2, r_k] with N(0, 1/(2 r_{k-1})) entries."""
    rng = np.random.default_rng(seed)
    d = len(ranks) - 1
    cores = []
    for k in range(d):
        s = scale if scale is not None else 1.0 / np.sqrt(2.0 * ranks[k])
        cores.append(rng.standard_normal((ranks[k], 2, 2, ranks[k + 1])) * s)
    return cores


def random_vector(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def mlp_init(layers, seed):
    """Initial MLP parameters [W1, b1, W2, b2, ...], W ~ U(+-sqrt(6/(fan_in+fan_out)))."""
    rng = np.random.default_rng(seed)
    params = []
    for fin, fout in zip(layers[:-1], layers[1:]):
        lim = np.sqrt(6.0 / (fin + fout))
        params.append(rng.uniform(-lim, lim, size=(fin, fout)))
        params.append(np.zeros(fout))
    return params
