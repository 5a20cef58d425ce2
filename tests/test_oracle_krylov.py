import numpy as np

from oracle import krylov
from tests import cases, helpers


def test_fgmres_matches_direct_solve():
    snap = cases.newton_snapshots("tiny_box")
    h = snap["result"].history[4]
    S, rhs, ref = h["S"], h["rhs"], h["dgamma"]
    dinv = 1.0 / S.diagonal()
    x, it, hist = krylov.fgmres(lambda v: S @ v, lambda v: dinv * v, rhs,
                                tol=1e-12, restart=20, maxit=2000)
    assert np.linalg.norm(rhs - S @ x) <= 1.01e-12 * np.linalg.norm(rhs)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)
    assert hist[-1] <= 1e-12
