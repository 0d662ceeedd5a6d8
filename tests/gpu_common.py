"""Helpers shared by the GPU parity tests (comparison against the oracle)."""
import math
import numpy as np

TERMS = (("exchange", 1), ("anisotropy", 2), ("zeeman", 4), ("demag_self", 8),
         ("demag_cross", 16))

# Relative L2 bars per term and film (also applied as max |error| / max |H|,
# so that an error confined to a window edge or halo row cannot hide in the
# norm).  float32: 1e-5 for every term and the force.  float64: 1e-10 for
# every term and the total field, except the cross term and the force
# (1e-9): their kernel entries are Newell's closed forms at 2 to 40 cells of
# displacement, where the 27-term difference cancels (r / cell)^6-fold and
# leaves 1e-8..1e-6 relative rounding error per entry that device and host
# realise differently (libm and summation order; both sides are equally
# accurate); the cross term is 1e-2..1e-3 of the total field, whose error
# stays below 3e-12.  Measured: cross term 1e-11..6e-10, force up to 7e-10.
TOL = {32: 1e-5, 64: 1e-10}
TOL_CROSS = {32: 1e-5, 64: 1e-9}


def max_rel(a, b):
    mb = np.abs(b).max()
    return np.abs(a - b).max() / mb if mb > 0 else np.abs(a).max()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def oracle_system(desc, drive, m, x_cells=None):
    from oracle.sim import System
    s = System(desc, drive, m)
    if x_cells is not None:
        s.x = x_cells * desc.dx
        s.s_int = int(math.floor(x_cells))
    return s
