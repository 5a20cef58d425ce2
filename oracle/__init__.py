"""CPU FP64 oracle for the QTT-accelerated PDIP Newton-step solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` use it.  It shares
no code with the HIP library; both read the seeded inputs of ``scenes``.

It is written to be checked against the paper by eye: plain NumPy/SciPy in
float64, each step in the order the paper (or the named textbook method it
follows) states it, no blocking, fusion or reordering.

Modules
-------
contacts  active set, contact frames, Morton ordering, slot map (Sec. 2.2, 3.3)
assembly  D, N = D^T M^-1 D, r = b + D^T M^-1 k, integration (Sec. 2.2-2.3)
pdip      primal-dual interior point on the conic QP, Schur complement (Sec. 2.4, 3.3)
tt        TT / QTT toolkit: Algorithm 1, matrix tensorisation, matvec, rounding,
          products, Newton-Schulz inverse (Sec. 3.1-3.2)
krylov    flexible GMRES with right preconditioning (Sec. 3.3, 4.2)
"""
