"""Pins for the local field terms."""
import numpy as np
import pytest
from workloads import Desc
from oracle.constants import MU0
from oracle.fields import exchange, anisotropy, zeeman


def test_helix_eigenvalue():
    d = Desc(n_films=1, nx=40, ny=3, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, Ms=8e5, Aex=1.3e-11)
    k = 2 * np.pi / (13 * d.dx)
    x = np.arange(d.nx) * d.dx
    m = np.zeros((3, 1, d.ny, d.nx))
    m[0] = np.cos(k * x)
    m[1] = np.sin(k * x)
    H = exchange(d, m)
    lam = 2 * d.Aex / (MU0 * d.Ms) * (2 * np.cos(k * d.dx) - 2) / d.dx ** 2
    assert np.allclose(H[:, :, :, 1:-1], lam * m[:, :, :, 1:-1], rtol=1e-12, atol=1e-6)
    # end cells see one neighbour only
    assert H[0, 0, 0, 0] == pytest.approx(2 * d.Aex / (MU0 * d.Ms) * (m[0, 0, 0, 1] - m[0, 0, 0, 0]) / d.dx ** 2)


def test_uniform_has_no_exchange():
    d = Desc(nx=6, ny=5, nz=3)
    m = np.zeros((3, 3, 5, 6))
    m[1] = 1
    assert np.abs(exchange(d, m)).max() == 0.0


def test_anisotropy_and_zeeman():
    d = Desc(Ku=5e5, Ms=1e6, u=(0, 0, 2.0), Hext=(1.0, -2.0, 3.0), nx=2, ny=2)
    m = np.zeros((3, 1, 2, 2))
    m[0] = 0.6
    m[2] = 0.8
    Ha = anisotropy(d, m)
    assert Ha[2, 0, 0, 0] == pytest.approx(2 * 5e5 / (MU0 * 1e6) * 0.8)
    assert Ha[0].max() == 0
    Hz = zeeman(d, m)
    assert Hz[:, 0, 1, 1].tolist() == [1.0, -2.0, 3.0]
