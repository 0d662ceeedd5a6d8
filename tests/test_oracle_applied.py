"""Pins of the non-uniform applied field in the moving magnet (Sec. II.A;
oracle/applied.py): properties that hold for the interpolant whatever its
implementation -- exact reproduction of uniform fields, of the lattice
values at integer offsets and of low-order polynomials, invariance under a
shift by one period, and the spline's approximation bound."""
import math
import numpy as np
import pytest

from workloads import Desc, Drive
from workloads.states import domain_state
from oracle import applied
from oracle.sim import System


def films(mode=0, pbc=0, nx=40, ny=6, travel=3):
    return Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=3, max_travel_cells=travel,
                Ms=8e5, Aex=1.3e-11, alpha=0.2, cross_mode=mode, pbc=pbc, pbc_images=1)


def frame_field(d, f):
    """(3, ny, width) from f(lattice x index, y index, component)."""
    W = 0 if d.pbc & 1 else d.max_travel_cells + d.halo
    xs = np.arange(applied.slider_width(d)) - W
    ys = np.arange(d.ny)
    X, Y = np.meshgrid(xs, ys)
    return np.array([f(X, Y, c) for c in range(3)], dtype=np.float64)


@pytest.mark.parametrize("mode", [0, 2])
def test_uniform_field_is_sampled_exactly(mode):
    d = films(mode)
    hs = frame_field(d, lambda X, Y, c: np.full(X.shape, 1e3 * (c + 1)))
    for x_cells in (-2.7, -0.5, 0.0, 0.31, 2.99):
        s_int = math.floor(x_cells)
        out = applied.slider_samples(d, hs, x_cells * d.dx, s_int)
        for c in range(3):
            assert np.allclose(out[c], 1e3 * (c + 1), rtol=1e-13, atol=0)


@pytest.mark.parametrize("mode", [0, 2])
def test_integer_offsets_take_the_lattice_values(mode):
    d = films(mode)
    rng = np.random.default_rng(3)
    hs = rng.standard_normal((3, d.ny, applied.slider_width(d)))
    W = d.max_travel_cells + d.halo
    for s in (-3, -1, 0, 2, 3):
        out = applied.slider_samples(d, hs, s * d.dx, s)
        assert np.allclose(out, hs[:, :, W + s:W + s + d.nx], rtol=0, atol=1e-12)


def test_linear_interpolation_reproduces_a_linear_field():
    d = films(2)
    hs = frame_field(d, lambda X, Y, c: 3.0 + 0.7 * X - 0.2 * Y + c)
    for x_cells in (-2.3, 0.45, 1.75):
        s_int = math.floor(x_cells)
        out = applied.slider_samples(d, hs, x_cells * d.dx, s_int)
        X = np.arange(d.nx)[None, :] + x_cells
        Y = np.arange(d.ny)[:, None]
        for c in range(3):
            assert np.allclose(out[c], 3.0 + 0.7 * X - 0.2 * Y + c, rtol=0, atol=1e-12)


def test_spline_reproduces_a_cubic_away_from_the_mirrored_ends():
    """The cubic B-spline interpolant reproduces cubics; the mirror
    extension of the window perturbs it by |z1|^j at j samples from an end
    (z1 = sqrt(3) - 2), so cells at least 12 samples inside agree to 1e-6."""
    d = films(0, nx=48)
    f = lambda X: 1.0 + 0.3 * X - 0.02 * X ** 2 + 0.0007 * X ** 3
    hs = frame_field(d, lambda X, Y, c: f(X.astype(np.float64)))
    x_cells = 1.37
    out = applied.slider_samples(d, hs, x_cells * d.dx, 1)
    X = np.arange(d.nx) + x_cells
    inner = slice(12 - d.halo, d.nx - 12 + d.halo)
    assert np.allclose(out[0][:, inner], f(X)[None, inner], rtol=0, atol=1e-6 * np.abs(f(X)).max())


def test_periodic_shift_by_one_period_is_invisible():
    d = films(0, pbc=1, nx=24)
    rng = np.random.default_rng(5)
    hs = rng.standard_normal((3, d.ny, d.nx))
    a = applied.slider_samples(d, hs, 0.4 * d.dx, 0)
    b = applied.slider_samples(d, hs, (0.4 + d.nx) * d.dx, d.nx)
    assert np.allclose(a, b, rtol=0, atol=1e-12)


def test_spline_of_a_smooth_sinusoid_within_its_error_bound():
    """f = sin(2 pi X / 16): the cubic spline's error is of order
    (pi / 8)^4 / 100 ~ 2e-4 of the amplitude for 16 samples per period
    (interior cells)."""
    d = films(0, nx=64)
    hs = frame_field(d, lambda X, Y, c: np.sin(2 * np.pi * X / 16.0))
    x_cells = 0.5
    out = applied.slider_samples(d, hs, x_cells * d.dx, 0)
    X = np.arange(d.nx) + x_cells
    inner = slice(8, d.nx - 8)
    err = np.abs(out[0][:, inner] - np.sin(2 * np.pi * X / 16.0)[None, inner]).max()
    assert err < 1e-3


def test_system_adds_the_applied_field_to_the_zeeman_term():
    d = films(0).replace(Hext=(1e2, 0.0, -3e2))
    m = [domain_state((1, d.ny, d.nx), 1), domain_state((1, d.ny, d.nx), 2)]
    s = System(d, Drive(x0=0.63 * d.dx), m)
    t0, _ = s.field_terms()
    rng = np.random.default_rng(7)
    hb = rng.standard_normal((3, d.ny, d.nx)) * 1e3
    hs = rng.standard_normal((3, d.ny, applied.slider_width(d))) * 1e3
    s.hext_fields = [hb, hs]
    t1, _ = s.field_terms()
    assert np.allclose(t1[0]["zeeman"] - t0[0]["zeeman"], hb[:, None], rtol=0, atol=1e-9)
    assert np.allclose(t1[1]["zeeman"] - t0[1]["zeeman"], applied.slider_samples(d, hs, s.x, s.s_int)[:, None],
                       rtol=0, atol=1e-9)
    for k in ("exchange", "anisotropy", "demag_self", "demag_cross"):
        assert np.array_equal(t1[1][k], t0[1][k])
