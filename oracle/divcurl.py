"""Divergence and curl of the interpolated stray field (Sec. IV.A, Eq. 13).

TEST INFRASTRUCTURE ONLY (part of the float64 oracle).

The base film's field, sampled inside the slider at the partial movement x,
has per slider cell i the two-point central-difference divergence and curl
    div_i  = sum_a (H_a(i + e_a) - H_a(i - e_a)) / (2 d_a)
    curl_i = (d_y H_z - d_z H_y, d_z H_x - d_x H_z, d_x H_y - d_y H_x)_i
from the field at the six neighbour points of the shifted lattice
(System.base_field_stencil), and Eq. 13 averages their magnitudes over the
N slider cells:
    D(x) = (1/N) sum_i |div_i|,    C(x) = (1/N) sum_i |curl_i|.
The study compares D and C at each x with the stationary, non-interpolated
values (x at a lattice position), for the spline of the direct field
(cross_mode 0), the scalar potential (cross_mode 1) and linear
interpolation of the field vectors (cross_mode 2).

(The potential mode's field is a four-point difference of one lattice
function; its two-point curl is small but not zero, since a two-point
difference along one axis does not commute with a four-point one along
another.)

Pins (tests/test_oracle_divcurl.py): a linear field H = A r gives exactly
D = |tr A| and C = |curl| of A; at lattice positions every interpolant
reproduces the stationary values; the paper's observation that linear
interpolation changes D one to two orders more than the spline does.
"""
import math
import numpy as np


def div_curl_cells(desc, st):
    """Per-cell divergence (ny, nx) and curl (3, ny, nx) from a stencil."""
    dx, dy, dz = desc.dx, desc.dy, desc.dz

    def d(a, key_p, key_m, h):
        return (st[key_p][a] - st[key_m][a]) / (2.0 * h)
    div = d(0, "xp", "xm", dx) + d(1, "yp", "ym", dy) + d(2, "zp", "zm", dz)
    curl = np.array([d(2, "yp", "ym", dy) - d(1, "zp", "zm", dz),
                     d(0, "zp", "zm", dz) - d(2, "xp", "xm", dx),
                     d(1, "xp", "xm", dx) - d(0, "yp", "ym", dy)])
    return div, curl


def div_curl(system, x):
    """(D(x), C(x)) of Eq. 13 for the base film's field in the slider at
    slider position x [m] (s_int = floor(x / dx))."""
    desc = system.desc
    s_int = int(math.floor(x / desc.dx))
    st = system.base_field_stencil(system.m[0], x, s_int)
    div, curl = div_curl_cells(desc, st)
    n = desc.nx * desc.ny
    return float(np.abs(div).sum() / n), float(np.sqrt((curl * curl).sum(axis=0)).sum() / n)


def relative_curve(system, xs):
    """(D(x) - D0) / D0 and (C(x) - C0) / C0 against the stationary field
    (the slider at x = 0)."""
    D0, C0 = div_curl(system, 0.0)
    out = []
    for x in xs:
        D, C = div_curl(system, x)
        out.append(((D - D0) / D0, (C - C0) / C0 if C0 > 0 else C))
    return out
