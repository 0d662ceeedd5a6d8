"""Non-uniform applied field in the moving magnet (Sec. II.A).

TEST INFRASTRUCTURE ONLY (part of the float64 oracle).

An applied field that varies in space moves with neither film: it is given
on the fixed lattice of the frame.  The base film's cells lie on that
lattice and take its values as they are.  The slider's cells, displaced by
the partial movement, take the field vectors interpolated directly along the
motion axis: an applied field is not in general a gradient, so it cannot go
through a scalar potential (Sec. II.A).  The interpolant is the one the
direct stray field uses (reading in the design notes): the prefiltered cubic
B-spline on the window of the slider's cells plus `halo` cells on each side,
with whole-sample mirror boundaries (cross_mode 0 and 1); linear
interpolation in the comparison mode (cross_mode 2).

Layout: film 0, (3, ny, nx) on its cells.  The slider's layer, (3, ny,
nx + 2 W) with W = max_travel_cells + halo; column c is lattice x index c - W.
With periodic x: (3, ny, nx), the period, indices taken modulo nx.

The force of Eq. 3 is the base film's field only; the applied field does not
enter it.

Pins (tests/test_oracle_applied.py):
- a uniform field is sampled exactly at every offset;
- at integer offsets the slider takes the lattice values;
- linear interpolation reproduces a field linear in x exactly;
- the spline reproduces a cubic in x away from the window's mirrored ends;
- a shift by one period of a periodic film leaves the samples unchanged;
- a smooth sinusoid is sampled within the spline's error bound.
"""
import numpy as np

from .spline import prefilter, interp_1d, linear_1d


def slider_width(desc):
    """Columns of the slider layer's applied-field array."""
    if desc.pbc & 1:
        return desc.nx
    return desc.nx + 2 * (desc.max_travel_cells + desc.halo)


def slider_samples(desc, hs, x, s_int):
    """The applied field at the slider's cells, (3, ny, nx), for slider
    position x [m] seated at lattice offset s_int."""
    nx, h = desc.nx, desc.halo
    hs = np.asarray(hs, dtype=np.float64)
    assert hs.shape == (3, desc.ny, slider_width(desc)), hs.shape
    cols = s_int - h + np.arange(nx + 2 * h)          # window: lattice columns
    if desc.pbc & 1:
        idx = np.mod(cols, nx)
    else:
        idx = cols + desc.max_travel_cells + h
        assert idx.min() >= 0 and idx.max() < hs.shape[-1], "slider beyond the applied field's columns"
    G = hs[:, :, idx]
    u = np.arange(nx, dtype=np.float64) + h + (x / desc.dx - s_int)
    if desc.cross_mode == 2:
        return linear_1d(G, u)
    return interp_1d(prefilter(G, axis=-1), u)
