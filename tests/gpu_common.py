"""Helpers shared by the GPU parity tests (comparison against the oracle)."""
import math
import numpy as np

TERMS = (("exchange", 1), ("anisotropy", 2), ("zeeman", 4), ("demag_self", 8),
         ("demag_cross", 16))

# Relative L2 bars.  float32: 1e-5, the bar set for the float32 path.  float64: FFT rounding of the
# float64 path is ~1e-15; the bar is set by the Newell kernel near the switch
# radius, where the independent float64 evaluations (device libm vs host
# libm) differ by ~1e-7 of entries that carry ~1e-4 of the field.
TOL = {32: 1e-5, 64: 1e-9}


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
