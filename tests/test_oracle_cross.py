"""Pins for the oracle's cross-film geometry (Sec. II.A, III.A, Eqs. 3, 6-8).

The two-film oracle (oracle.sim.System) builds the other film's field on
lattice windows: the slider layer z_s, rows -1..ny, the force layers
z_s +- 1, the mirrored layer -z_s for the slider's field on the base, and
in potential mode the potential on layers and rows around them.  At an
integer offset (x_p = 0) the spline reproduces the window data exactly, so
every sampled field, and the force of Eq. 3, must equal a brute-force sum
over source cells written here from the physical cell centres alone:
base cell (i, j) at ((i+1/2) dx, (j+1/2) dy, dz/2), slider cell at
(x_s + (i+1/2) dx, (j+1/2) dy, (gap + 1 + 1/2) dz).  Nothing below reuses
the oracle's window boxes, its FFT sums or its stencil helper.

Each pin is also run against planted mistakes (a layer, row, offset-sign
or stencil slip in a patched copy of the oracle) and must reject them.
"""
import math
import numpy as np
import pytest
from workloads import Desc, Drive
from workloads.states import random_unit
from oracle.constants import MU0
from oracle.newell import tensor_matrix
from oracle.potential_kernel import potential_kernel
from oracle import sim as oracle_sim
from oracle.sim import System, FROZEN


def films(nx=7, ny=5, gap=1, cross_mode=0, seed=3):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=3e-9, dz=2.5e-9,
             gap_cells=gap, Ms=9e5, cross_mode=cross_mode, halo=4)
    rng = np.random.default_rng(seed)
    m = [random_unit((1, ny, nx), rng) for _ in range(2)]
    return d, m


def centres(d, x_shift=0.0, layer=0):
    """Cell-centre coordinates (X, Y, Z) of a film, shape (ny, nx)."""
    jj, ii = np.meshgrid(np.arange(d.ny), np.arange(d.nx), indexing="ij")
    return ((ii + 0.5) * d.dx + x_shift, (jj + 0.5) * d.dy,
            np.full(ii.shape, (layer + 0.5) * d.dz))


def tensor_field_at(d, P, src_m, src_x_shift, src_layer):
    """H(P) = -Ms sum_j N(P - r_j) m_j over the source film's cells."""
    Xs, Ys, Zs = centres(d, src_x_shift, src_layer)
    out = np.zeros(3)
    N = tensor_matrix(P[0] - Xs, P[1] - Ys, P[2] - Zs, d.dx, d.dy, d.dz,
                      d.rc_cells)                       # (3, 3, ny, nx)
    for a in range(3):
        for b in range(3):
            out[a] -= d.Ms * np.sum(N[a, b] * src_m[b, 0])
    return out


def potential_at(d, P, src_m, src_x_shift, src_layer):
    """phi(P) = Ms sum_j S(P - r_j) . m_j over the source film's cells."""
    Xs, Ys, Zs = centres(d, src_x_shift, src_layer)
    S = potential_kernel(P[0] - Xs, P[1] - Ys, P[2] - Zs, d.dx, d.dy, d.dz)
    return d.Ms * sum(np.sum(S[b] * src_m[b, 0]) for b in range(3))


def grad4(fun, P, steps):
    """-grad by fourth-order central differences, written out per axis."""
    H = np.zeros(3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = steps[a]
        H[a] = -(fun(P - 2 * e) - 8 * fun(P - e) + 8 * fun(P + e)
                 - fun(P + 2 * e)) / (12 * steps[a])
    return H


def brute_force(d, m, s_int, potential=False):
    """(H on base, H on slider, F) at x_s = s_int dx by brute force."""
    mb, ms = m
    zs = d.gap_cells + 1
    xs = s_int * d.dx
    steps = np.array([d.dx, d.dy, d.dz])
    if potential:
        def base_field(P):
            return grad4(lambda Q: potential_at(d, Q, mb, 0.0, 0), P, steps)

        def slider_field(P):
            return grad4(lambda Q: potential_at(d, Q, ms, xs, zs), P, steps)
    else:
        def base_field(P):
            return tensor_field_at(d, P, mb, 0.0, 0)

        def slider_field(P):
            return tensor_field_at(d, P, ms, xs, zs)
    Hs = np.zeros((3, 1, d.ny, d.nx))
    Hb = np.zeros((3, 1, d.ny, d.nx))
    F = np.zeros(3)
    V = d.dx * d.dy * d.dz
    for j in range(d.ny):
        for i in range(d.nx):
            Ps = np.array([xs + (i + 0.5) * d.dx, (j + 0.5) * d.dy, (zs + 0.5) * d.dz])
            Pb = np.array([(i + 0.5) * d.dx, (j + 0.5) * d.dy, 0.5 * d.dz])
            Hs[:, 0, j, i] = base_field(Ps)
            Hb[:, 0, j, i] = slider_field(Pb)
            # Eq. 3: (m . grad) H with two-point central differences
            mi = ms[:, 0, j, i]
            for a in range(3):
                e = np.zeros(3)
                e[a] = steps[a]
                dH = (base_field(Ps + e) - base_field(Ps - e)) / (2 * steps[a])
                F += MU0 * d.Ms * V * mi[a] * dH
    return Hb, Hs, F


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def oracle_fields(d, m, s_int):
    s = System(d, Drive(mode=FROZEN, x0=s_int * d.dx), m)
    return s.cross_fields(m[0], m[1], s_int * d.dx, s_int)


@pytest.mark.parametrize("s_int", [0, 2, -1])
def test_direct_cross_fields_equal_brute_force(s_int):
    d, m = films()
    Hb, Hs, F = oracle_fields(d, m, s_int)
    rb, rs, rf = brute_force(d, m, s_int)
    assert rel(Hs, rs) < 1e-10
    assert rel(Hb, rb) < 1e-10
    assert rel(F, rf) < 1e-10


@pytest.mark.parametrize("s_int", [0, 1])
def test_potential_cross_fields_equal_brute_force(s_int):
    d, m = films(nx=6, ny=5, gap=3, cross_mode=1, seed=5)
    Hb, Hs, F = oracle_fields(d, m, s_int)
    rb, rs, rf = brute_force(d, m, s_int, potential=True)
    assert rel(Hs, rs) < 1e-10
    assert rel(Hb, rb) < 1e-10
    assert rel(F, rf) < 1e-9


# ---------------------------------------------------------------- mutations
# Each planted mistake lives in a patched copy of the oracle (monkeypatch),
# and the brute-force comparison above must reject it.

def _shift_box(dz=0, dy=0, sign=1):
    orig = System.cross_box

    def patched(self, direction, s_int):
        x0, nwx, y0, nwy, z0, nwz = orig(self, direction, sign * s_int)
        if direction == "b2s":
            return (x0, nwx, y0 + dy, nwy, z0 + dz, nwz)
        return (x0, nwx, y0, nwy, z0, nwz)
    return patched


@pytest.mark.parametrize("name,patch", [
    ("slider layer +1", dict(dz=1)),
    ("slider layer -1", dict(dz=-1)),
    ("one-row slip", dict(dy=1)),
    ("offset sign", dict(sign=-1)),
])
def test_direct_pin_rejects_geometry_slips(monkeypatch, name, patch):
    d, m = films()
    s_int = 2
    rb, rs, rf = brute_force(d, m, s_int)
    monkeypatch.setattr(System, "cross_box", _shift_box(**patch))
    Hb, Hs, F = oracle_fields(d, m, s_int)
    assert max(rel(Hs, rs), rel(Hb, rb), rel(F, rf)) > 1e-3, name


def test_direct_pin_rejects_mirrored_base_layer(monkeypatch):
    d, m = films()
    orig = System.cross_box

    def patched(self, direction, s_int):
        box = orig(self, direction, s_int)
        if direction == "s2b":
            x0, nwx, y0, nwy, z0, nwz = box
            return (x0, nwx, y0, nwy, -z0, nwz)    # +z_s instead of -z_s
        return box
    rb, rs, rf = brute_force(d, m, 0)
    monkeypatch.setattr(System, "cross_box", patched)
    Hb, Hs, F = oracle_fields(d, m, 0)
    assert rel(Hb, rb) > 1e-3


def test_potential_pin_rejects_two_point_stencil(monkeypatch):
    d, m = films(nx=6, ny=5, gap=3, cross_mode=1, seed=5)
    rb, rs, rf = brute_force(d, m, 0, potential=True)
    monkeypatch.setattr(oracle_sim, "_d4",
                        lambda fm2, fm1, fp1, fp2, h: (fp1 - fm1) / (2.0 * h))
    Hb, Hs, F = oracle_fields(d, m, 0)
    assert max(rel(Hs, rs), rel(Hb, rb)) > 1e-4


def test_potential_pin_rejects_row_slip(monkeypatch):
    d, m = films(nx=6, ny=5, gap=3, cross_mode=1, seed=5)
    rb, rs, rf = brute_force(d, m, 0, potential=True)
    monkeypatch.setattr(System, "cross_box", _shift_box(dy=1))
    Hb, Hs, F = oracle_fields(d, m, 0)
    assert rel(Hs, rs) > 1e-3
