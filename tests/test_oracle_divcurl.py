"""Pins for the oracle's divergence / curl study (Sec. IV.A, Eq. 13)."""
import math
import numpy as np
import pytest
from workloads import Desc, Drive
from workloads.states import random_unit
from oracle import divcurl
from oracle.sim import System, FROZEN


def films(mode, gap=3, nx=20, ny=14, seed=9):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=4e-9, dy=4e-9, dz=4e-9, gap_cells=gap, Ms=8e5,
             cross_mode=mode, max_travel_cells=2)
    rng = np.random.default_rng(seed)
    m = [random_unit((1, ny, nx), rng), random_unit((1, ny, nx), rng)]
    return System(d, Drive(mode=FROZEN), m)


def test_linear_field_closed_form():
    d = Desc(n_films=2, nx=5, ny=4, nz=1, dx=2e-9, dy=3e-9, dz=2.5e-9)
    A = np.array([[1.0, 2.0, -1.5], [0.5, -3.0, 4.0], [2.5, 1.0, 0.7]])
    jj, ii = np.meshgrid(np.arange(4), np.arange(5), indexing="ij")
    r = lambda ox, oy, oz: np.array([(ii + ox) * d.dx, (jj + oy) * d.dy, np.full(ii.shape, oz * d.dz)])
    field = lambda ox, oy, oz: np.einsum("ab,b...->a...", A, r(ox, oy, oz))
    st = {"c": field(0, 0, 0), "xp": field(1, 0, 0), "xm": field(-1, 0, 0), "yp": field(0, 1, 0),
          "ym": field(0, -1, 0), "zp": field(0, 0, 1), "zm": field(0, 0, -1)}
    div, curl = divcurl.div_curl_cells(d, st)
    assert np.allclose(div, np.trace(A), rtol=1e-13, atol=0)
    ref = np.array([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    assert np.allclose(curl, ref[:, None, None], rtol=1e-13, atol=0)


@pytest.mark.parametrize("mode", [0, 2])
def test_lattice_positions_reproduce_the_stationary_values(mode):
    s = films(mode)
    D0, C0 = divcurl.div_curl(s, 0.0)
    sp = films(0)
    assert (D0, C0) == pytest.approx(divcurl.div_curl(sp, 0.0), rel=1e-12)
    # a full cell with s_int held at 0 equals the re-seated lattice position
    st0 = s.base_field_stencil(s.m[0], 1.0 * s.desc.dx, 0)
    st1 = s.base_field_stencil(s.m[0], 1.0 * s.desc.dx, 1)
    for k in st0:
        inner = (slice(None), slice(None), slice(4, -4))
        assert np.abs(st0[k][inner] - st1[k][inner]).max() < 1e-9 * np.abs(st1[k]).max()


def test_linear_interpolation_changes_divergence_far_more_than_the_spline():
    # Sec. IV.A: random frozen base, slider 5 cells (20 nm) above; linear
    # interpolation moves D by percents, several times more than the spline
    # (measured here on 24 x 16 films: spline 0.7-1.1 %, linear 5.6-7.7 %)
    xs = [0.25, 0.5, 0.75]
    spl = divcurl.relative_curve(films(0, gap=5, nx=24, ny=16), [x * 4e-9 for x in xs])
    lin = divcurl.relative_curve(films(2, gap=5, nx=24, ny=16), [x * 4e-9 for x in xs])
    print("spline", spl, "linear", lin)
    for a, b in zip(spl, lin):
        assert abs(b[0]) > 3 * abs(a[0]) and abs(b[1]) > 3 * abs(a[1])
        assert abs(b[0]) > 1e-2
