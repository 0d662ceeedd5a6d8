"""Pins for the scalar-potential mode in films periodic in plane (Sec. III.A
end: the potential's values past the domain are copies from the other side;
Eqs. 7-8; the force of Eq. 3)."""
import numpy as np
import pytest
from workloads import Desc, Drive
from workloads.states import random_unit
from oracle.constants import MU0
from oracle.periodic import FilmPotWindow, brute_force_pot, periodic_s
from oracle.sim import System, FROZEN
from oracle.slab import SlabSystem


def films(pbc, nx=6, ny=4, nz=2, gap=3, seed=1, P=1):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=nz, dx=2e-9, dy=3e-9, dz=2.5e-9, gap_cells=gap, Ms=9e5, halo=4,
             max_travel_cells=4, cross_mode=1, pbc=pbc, pbc_images=P)
    rng = np.random.default_rng(seed)
    return d, [random_unit((nz, ny, nx), rng) for _ in range(2)]


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("pbc", [1, 2, 3])
@pytest.mark.parametrize("box,dz", [((0, 4, 0, 4), 2), ((-3, 9, -2, 7), -3), ((5, 3, 3, 2), 4)])
def test_potential_window_equals_brute_force_over_images(pbc, box, dz):
    d, _ = films(pbc, nx=4, ny=4, nz=1, P=2)
    m = random_unit((1, 4, 4), np.random.default_rng(pbc + 5 * abs(dz)))
    W = FilmPotWindow(d, *box, dz)(m)
    B = brute_force_pot(d, m, *box, dz)
    assert rel(W, B) < 1e-12


def potential_box(d, src, X0, nX, Y0, nY, Z0, nZ):
    """phi on the lattice points (X, Y, Z) of a box (cells, relative to the
    source film's lattice origin) by the direct sum over the source's cells,
    each displacement's image-summed kernel from periodic_s."""
    nz, ny, nx = src.shape[1:]
    DX = np.arange(X0 - (nx - 1), X0 + nX)
    DY = np.arange(Y0 - (ny - 1), Y0 + nY)
    GY, GX = np.meshgrid(DY, DX, indexing="ij")
    tab = {}
    for dz in range(Z0 - (nz - 1), Z0 + nZ):
        tab[dz] = [periodic_s(d, b, GX, GY, dz) for b in range(3)]
    phi = np.zeros((nZ, nY, nX))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for t in range(nZ):
                    T = tab[Z0 + t - k]
                    # rows Y - j, columns X - i of the displacement tables
                    r0, c0 = Y0 - j - DY[0], X0 - i - DX[0]
                    for b in range(3):
                        phi[t] += d.Ms * src[b, k, j, i] * T[b][r0:r0 + nY, c0:c0 + nX]
    return phi


def neg_grad4(phi, steps):
    """-grad by four-point central differences on the interior of a box
    padded by two points on each side: (3, nZ - 4, nY - 4, nX - 4)."""
    out = []
    for axis, h in zip((0, 1, 2), steps):
        n = phi.shape[axis]
        sl = lambda a, b: tuple(slice(a, n - b) if ax == axis else slice(2, phi.shape[ax] - 2) for ax in range(3))
        out.append(-(phi[sl(0, 4)] - 8 * phi[sl(1, 3)] + 8 * phi[sl(3, 1)] - phi[sl(4, 0)]) / (12 * h))
    return np.array(out)


@pytest.mark.parametrize("pbc,nz,s_int", [(1, 2, 0), (3, 2, 7), (2, 1, 2), (3, 3, -1)])
def test_periodic_potential_mode_equals_brute_force(pbc, nz, s_int):
    """At integer offsets (one beyond the period): each film's cross field is
    the four-point difference of the directly summed periodic potential of
    the other, and Eq. 3's force the two-point difference of the base's field
    on the slider's stencil."""
    d, m = films(pbc, nz=nz, seed=3 * pbc + nz)
    s = SlabSystem(d, Drive(mode=FROZEN, x0=s_int * d.dx), m)
    Hb, Hs, F = s.cross_fields(m[0], m[1], s_int * d.dx, s_int)
    zs = d.nz + d.gap_cells
    steps = (d.dz, d.dy, d.dx)
    # base potential around the slider's cells and their stencil (+-1), padded by 2
    phb = potential_box(d, m[0], s_int - 3, d.nx + 6, -3, d.ny + 6, zs - 3, d.nz + 6)
    Hgrid = neg_grad4(phb, steps)                      # points (zs-1.., -1.., s_int-1..)
    Hgrid = Hgrid[[2, 1, 0]]                           # components x, y, z
    rs = Hgrid[:, 1:-1, 1:-1, 1:-1]
    assert rel(Hs, rs) < 1e-9
    V = d.dx * d.dy * d.dz
    dH = [(Hgrid[:, 1:-1, 1:-1, 2:] - Hgrid[:, 1:-1, 1:-1, :-2]) / (2 * d.dx),
          (Hgrid[:, 1:-1, 2:, 1:-1] - Hgrid[:, 1:-1, :-2, 1:-1]) / (2 * d.dy),
          (Hgrid[:, 2:, 1:-1, 1:-1] - Hgrid[:, :-2, 1:-1, 1:-1]) / (2 * d.dz)]
    rF = MU0 * d.Ms * V * sum((m[1][a][None] * dH[a]).sum(axis=(1, 2, 3)) for a in range(3))
    assert np.abs(F - rF).max() < 1e-8 * np.abs(rF).max()
    # the slider's potential on the base's cells (slider lattice coordinates)
    phs = potential_box(d, m[1], -s_int - 2, d.nx + 4, -2, d.ny + 4, -zs - 2, d.nz + 4)
    rb = neg_grad4(phs, steps)[[2, 1, 0]]
    assert rel(Hb, rb) < 1e-9


@pytest.mark.parametrize("pbc", [1, 2, 3])
def test_periodic_potential_one_layer_thick_equals_film_oracle(pbc):
    """One-layer films: the thick-film oracle's periodic potential mode is the
    film oracle's at a fractional offset (the same windows and copies)."""
    d, m = films(pbc, nx=8, ny=6, nz=1, seed=pbc)
    x = 1.37 * d.dx
    a = SlabSystem(d, Drive(mode=FROZEN, x0=x), m).cross_fields(m[0], m[1], x, 1)
    b = System(d, Drive(mode=FROZEN, x0=x), m).cross_fields(m[0], m[1], x, 1)
    for u, v in zip(a, b):
        assert rel(u, v) < 1e-12


def test_periodic_potential_mode_physics():
    """A uniform magnetisation gives each film the same cross field in every
    cell of a layer (translation invariance along both periods), and a shift
    of the slider by one period changes neither field nor force."""
    d, m = films(3, nx=6, ny=4, nz=2, seed=9)
    up = [np.tile(np.array([0.3, -0.1, 0.95])[:, None, None, None], (1, 2, 4, 6))] * 2
    x = 1.3 * d.dx
    Hb, Hs, _ = SlabSystem(d, Drive(mode=FROZEN, x0=x), up).cross_fields(up[0], up[1], x, 1)
    for h in (Hb, Hs):
        assert np.abs(h - h[:, :, :1, :1]).max() < 1e-9 * np.abs(h).max()
    a = SlabSystem(d, Drive(mode=FROZEN, x0=x), m).cross_fields(m[0], m[1], x, 1)
    b = SlabSystem(d, Drive(mode=FROZEN, x0=x + d.nx * d.dx), m).cross_fields(m[0], m[1], x + d.nx * d.dx,
                                                                              1 + d.nx)
    for u, v in zip(a, b):
        assert rel(u, v) < 1e-12
