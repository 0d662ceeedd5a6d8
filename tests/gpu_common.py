"""Helpers shared by the GPU parity tests (comparison against the oracle)."""
import math
import numpy as np

TERMS = (("exchange", 1), ("anisotropy", 2), ("zeeman", 4), ("demag_self", 8),
         ("demag_cross", 16))

# Relative L2 bars per term and film (also applied as max |error| / max |H|,
# so that an error confined to a window edge or halo row cannot hide in the
# norm).  float32: 1e-5.  float64: 1e-10; FFT rounding of the float64 path is
# ~1e-15, and the Newell entries near the switch radius, where device and
# host libm differ after the cancellation, carry ~1e-4 of the field.
TOL = {32: 1e-5, 64: 1e-10}


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
