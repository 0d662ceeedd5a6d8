"""Pins for the lattice sums of Eqs. (6)-(7): FFT route vs brute force."""
import numpy as np
import pytest
from workloads import Desc
from oracle.convolution import (demag_window, potential_window, direct_sum,
                                demag_kernel_fn, potential_kernel_fn)


def small_desc(**kw):
    d = Desc(n_films=2, nx=5, ny=4, nz=1, dx=2e-9, dy=3e-9, dz=2.5e-9, Ms=8e5,
             rc_cells=3.0)
    return d.replace(**kw)


@pytest.mark.parametrize("box", [(0, 5, 0, 4, 0, 1), (-4, 13, -1, 6, 1, 3), (2, 9, 0, 4, -2, 1)])
def test_fft_window_equals_direct(box):
    d = small_desc()
    rng = np.random.default_rng(5)
    m = rng.standard_normal((3, 1, 4, 5))
    fast = demag_window(d, box)(m)
    slow = direct_sum(demag_kernel_fn(d), d, m, box)
    assert np.allclose(fast, slow, rtol=0, atol=1e-12 * np.abs(slow).max())
    pf = potential_window(d, box)(m)
    ps = direct_sum(potential_kernel_fn(d), d, m, box)
    assert np.allclose(pf, ps, rtol=0, atol=1e-12 * np.abs(ps).max())


def test_uniform_cube_average_is_third():
    n = 4
    d = Desc(n_films=1, nx=n, ny=n, nz=n, dx=1e-9, dy=1e-9, dz=1e-9, Ms=1.0)
    m = np.zeros((3, n, n, n))
    m[2] = 1.0
    H = demag_window(d, (0, n, 0, n, 0, n))(m)
    assert H[2].mean() == pytest.approx(-1.0 / 3.0, abs=1e-13)
    assert abs(H[0].mean()) < 1e-14


def test_3d_window_direct():
    d = Desc(n_films=1, nx=3, ny=2, nz=3, dx=1e-9, dy=1e-9, dz=1e-9, Ms=2.0,
             rc_cells=2.5)
    rng = np.random.default_rng(7)
    m = rng.standard_normal((3, 3, 2, 3))
    box = (0, 3, 0, 2, 0, 3)
    assert np.allclose(demag_window(d, box)(m),
                       direct_sum(demag_kernel_fn(d), d, m, box), atol=1e-12)
