"""Pins for the periodic in-plane boundaries of the oracle (Sec. III.A end,
Sec. IV.B): wrapped kernel sums, periodic windows, periodic exchange."""
import math
import numpy as np
import pytest
from workloads import Desc, Drive
from workloads.states import random_unit, domain_state
from oracle.periodic import FilmWindow, BoxWindow, brute_force, exchange_periodic
from oracle.constants import MU0
from oracle.sim import System, FROZEN


def film(pbc, P=2, nx=6, ny=4, **kw):
    return Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=3e-9, dz=2.5e-9, Ms=9e5, pbc=pbc,
                pbc_images=P, **kw)


@pytest.mark.parametrize("pbc", [1, 2, 3])
@pytest.mark.parametrize("box", [(0, 6, 0, 4, 0), (-3, 10, -1, 6, 2), (5, 4, 2, 3, -2)])
def test_fft_route_equals_brute_force_over_images(pbc, box):
    d = film(pbc)
    m = random_unit((1, 4, 6), np.random.default_rng(pbc))
    W = FilmWindow(d, *box)(m)
    B = brute_force(d, m, *box)
    assert np.abs(W - B).max() < 1e-13 * np.abs(B).max()


def prism_centre_field(a, b, c):
    """-H/Ms at the centre of a uniformly magnetised a x b x c prism along c
    (textbook closed form; a cube gives 1/3)."""
    return 2.0 / math.pi * math.atan(a * b / (c * math.sqrt(a * a + b * b + c * c)))


def test_prism_centre_formula_cube():
    assert prism_centre_field(1.0, 1.0, 1.0) == pytest.approx(1.0 / 3.0, rel=1e-15)


@pytest.mark.parametrize("P", [8, 32])
def test_uniform_periodic_film_is_the_image_prism(P):
    # both axes periodic: every cell sees the same (2P+1) n x (2P+1) n plate
    # of the film centred on itself; its field is the prism's centre field
    n, t = 8, 2e-9
    d = Desc(n_films=1, nx=n, ny=n, nz=1, dx=t, dy=t, dz=t, Ms=1e6, pbc=3, pbc_images=P)
    S = (2 * P + 1) * n * t
    for comp, (a, b, c) in ((2, (S, S, t)), (0, (S, t, S))):
        m = np.zeros((3, 1, n, n))
        m[comp] = 1.0
        H = FilmWindow(d, 0, n, 0, n, 0)(m)
        assert np.ptp(H[comp]) < 1e-12 * d.Ms      # the same in every cell
        others = [c for c in range(3) if c != comp]
        assert np.abs(H[others]).max() < 1e-12 * d.Ms
        ref = -d.Ms * prism_centre_field(a, b, c)
        assert H[comp].mean() == pytest.approx(ref, rel=2e-3)


def test_uniform_film_periodic_in_x_is_uniform_along_x():
    d = film(1, P=3, nx=8, ny=5)
    m = np.zeros((3, 1, 5, 8))
    m[1] = 1.0
    H = FilmWindow(d, 0, 8, 0, 5, 0)(m)
    assert np.abs(H - H[..., :1]).max() < 1e-12 * np.abs(H).max()


def test_slider_shifted_by_one_period_sees_the_same_fields():
    d = film(1, P=2, nx=10, ny=6).replace(gap_cells=1, max_travel_cells=12)
    m = [domain_state((1, 6, 10), 7), domain_state((1, 6, 10), 8)]
    s = System(d, Drive(mode=FROZEN), m)
    a = s.cross_fields(*m, 0.3 * d.dx, 0)
    b = s.cross_fields(*m, (0.3 + d.nx) * d.dx, d.nx)
    for u, v in zip(a, b):
        assert np.abs(np.asarray(u) - np.asarray(v)).max() <= 1e-12 * max(np.abs(u).max(), 1e-300)


def test_periodic_window_halo_is_a_copy():
    d = film(3, P=1, nx=6, ny=4)
    m = random_unit((1, 4, 6), np.random.default_rng(2))
    W = BoxWindow(d, (-4, 14, -1, 6, 2, 1))(m)
    # column x and x + 6, row y and y + 4 are the same lattice point
    assert np.abs(W[..., :, 0:8] - W[..., :, 6:14]).max() == 0.0
    assert np.abs(W[..., 0:2, :] - W[..., 4:6, :]).max() == 0.0


def test_periodic_exchange_helix_everywhere():
    nx, q = 16, 3
    d = Desc(n_films=1, nx=nx, ny=3, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, Ms=8e5, Aex=1.3e-11, pbc=1)
    k = 2 * math.pi * q / (nx * d.dx)
    x = (np.arange(nx) + 0.5) * d.dx
    m = np.zeros((3, 1, 3, nx))
    m[0] = np.cos(k * x)
    m[1] = np.sin(k * x)
    H = exchange_periodic(d, m)
    lam = 2 * d.Aex / (MU0 * d.Ms) * (2 * math.cos(k * d.dx) - 2) / d.dx ** 2
    assert np.abs(H - lam * m).max() < 1e-9 * abs(lam)
