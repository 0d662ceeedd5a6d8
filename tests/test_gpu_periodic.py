"""Periodic in-plane boundaries (Sec. III.A end, Sec. IV.B) on the GPU
against the float64 oracle (oracle/periodic.py): every field term and the
force of Eq. 3 for films periodic in x, y or both, with the slider inside
and beyond the first period, and RK4 trajectories whose slider crosses the
period boundary."""
import numpy as np
import pytest

from workloads import Desc, Drive, slider_mass_damping
from workloads.states import domain_state
from test_gpu_parity import check_fields
from test_gpu_steps import track

pytestmark = pytest.mark.gpu


def films(pbc, prec, nx=48, ny=20, images=3, cross_mode=0, gap=1):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=gap, max_travel_cells=2,
             Ms=1.1e6, Aex=1.5e-11, alpha=0.1, Ku=8e5, u=(0.1, 0.0, 1.0), Hext=(2e3, -1e3, 5e3),
             precision=prec, pbc=pbc, pbc_images=images, cross_mode=cross_mode)
    m = [domain_state((1, ny, nx), 61), domain_state((1, ny, nx), 62)]
    return d, m


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("pbc", [1, 2, 3])
def test_periodic_fields_and_force(pbc, prec):
    d, m = films(pbc, prec)
    check_fields(d, Drive(), m, x_cells=1.37)
    if pbc & 1:
        # beyond the sized travel: the window wraps around the period
        check_fields(d, Drive(), m, x_cells=d.nx + 0.4)
        check_fields(d, Drive(), m, x_cells=-3.6)


@pytest.mark.parametrize("prec", [32, 64])
def test_periodic_ragged_and_single_film(prec):
    d, m = films(3, prec, nx=30, ny=9, images=1)
    check_fields(d, Drive(), m, x_cells=0.5)
    d1 = d.replace(n_films=1)
    check_fields(d1, Drive(), m[:1])


@pytest.mark.parametrize("prec", [32, 64])
def test_slider_crosses_the_period(prec):
    """Velocity drive at 5 m/s from 0.02 cell before the period's end: the
    slider re-seats into the next period (s_int = nx) after 80 steps."""
    d, m = films(3, prec)
    x0 = (d.nx - 0.02) * d.dx
    seats, worst = track(d, Drive(mode=1, v_d=5.0, x0=x0), m, 1e-13, 200)
    assert seats == {d.nx - 1, d.nx}


def test_spring_drive_on_periodic_films_fp32():
    d, m = films(3, 32)
    mass, gv = slider_mass_damping(d.nx, d.ny, 1e-3)
    x0 = 0.98 * d.dx
    drv = Drive(mode=2, v_d=5.0, k=1e-3, mass=mass, gamma_v=gv, x_anchor0=x0, x0=x0, v0=5.0)
    seats, worst = track(d, drv, m, 1e-13, 200)
    assert 1 in seats


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("pbc", [1, 2, 3])
def test_periodic_potential_mode_fields_and_force(pbc, prec):
    """Scalar-potential mode (gap 3) on periodic films: the potential's
    window rows and columns past the period are the other side's (Sec. III.A
    end), sampled and differenced as on open films."""
    print(f"periodic potential pbc={pbc} p{prec}", flush=True)
    d, m = films(pbc, prec, cross_mode=1, gap=3)
    check_fields(d, Drive(), m, x_cells=1.37)
    if pbc & 1:
        check_fields(d, Drive(), m, x_cells=d.nx + 0.4)
        check_fields(d, Drive(), m, x_cells=-3.6)


@pytest.mark.parametrize("prec", [32, 64])
def test_periodic_potential_and_linear_ragged(prec):
    """Ragged periods (nx = 30, ny = 9) in the potential mode and with the
    linear interpolant (cross_mode 2)."""
    print(f"periodic ragged potential/linear p{prec}", flush=True)
    d, m = films(3, prec, nx=30, ny=9, images=1, cross_mode=1, gap=3)
    check_fields(d, Drive(), m, x_cells=0.5)
    d, m = films(3, prec, nx=30, ny=9, images=1, cross_mode=2)
    check_fields(d, Drive(), m, x_cells=-0.7)


@pytest.mark.parametrize("prec", [32, 64])
def test_periodic_potential_slider_crosses_the_period(prec):
    """Potential mode: a velocity drive re-seats the slider into the next
    period, compared with the oracle's trajectory along the way."""
    print(f"periodic potential crossing p{prec}", flush=True)
    d, m = films(3, prec, cross_mode=1, gap=3)
    x0 = (d.nx - 0.02) * d.dx
    seats, worst = track(d, Drive(mode=1, v_d=5.0, x0=x0), m, 1e-13, 200)
    assert seats == {d.nx - 1, d.nx}
