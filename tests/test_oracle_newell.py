"""Pins for the oracle's demagnetising tensor (Eq. 6, Newell et al.)."""
import numpy as np
import pytest
from oracle import newell
from oracle.newell import demag_tensor, newell_exact, dipole


def aharoni_dz(a, b, c):
    """Magnetometric demag factor along c of a 2a x 2b x 2c prism.

    A. Aharoni, J. Appl. Phys. 83, 3432 (1998), Eq. (1) -- an independent
    closed form (not derived from Newell's f, g).
    """
    r = np.sqrt(a * a + b * b + c * c)
    rab, rbc, rac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    t = ((b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
         + b / (2 * c) * np.log((rab + a) / (rab - a))
         + a / (2 * c) * np.log((rab + b) / (rab - b))
         + c / (2 * a) * np.log((rbc - b) / (rbc + b))
         + c / (2 * b) * np.log((rac - a) / (rac + a))
         + 2 * np.arctan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (rac + rbc)
         - (rab ** 3 + rbc ** 3 + rac ** 3) / (3 * a * b * c))
    return t / np.pi


def test_aharoni_formula_sanity():
    assert aharoni_dz(1, 1, 1) == pytest.approx(1 / 3, abs=1e-14)
    a, b, c = 1.0, 2.0, 3.5
    s = aharoni_dz(b, c, a) + aharoni_dz(c, a, b) + aharoni_dz(a, b, c)
    assert s == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("cell", [(1.0, 1.0, 1.0), (1.0, 2.0, 3.0), (2e-9, 2e-9, 5e-9)])
def test_trace_is_one_at_origin(cell):
    tr = sum(newell_exact(c, 0.0, 0.0, 0.0, *cell) for c in ("xx", "yy", "zz"))
    assert tr == pytest.approx(1.0, abs=1e-12)


def test_cube_self_factor():
    for c in ("xx", "yy", "zz"):
        assert newell_exact(c, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0) == pytest.approx(1 / 3, abs=1e-14)
    for c in ("xy", "xz", "yz"):
        assert abs(newell_exact(c, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0)) < 1e-15


def test_single_cell_equals_prism_factor():
    dx, dy, dz = 1.0, 2.0, 3.0
    assert newell_exact("zz", 0, 0, 0, dx, dy, dz) == pytest.approx(
        aharoni_dz(dx / 2, dy / 2, dz / 2), rel=1e-12)
    assert newell_exact("xx", 0, 0, 0, dx, dy, dz) == pytest.approx(
        aharoni_dz(dy / 2, dz / 2, dx / 2), rel=1e-12)


@pytest.mark.parametrize("n", [(3, 4, 5), (2, 3, 1)])
def test_block_average_equals_aharoni(n):
    """(1/ncells) sum_ij N(r_i - r_j) over a block = the block's demag factor."""
    nx, ny, nz = n
    d = (1.0, 1.3, 0.7)
    ix = np.arange(-(nx - 1), nx)
    iy = np.arange(-(ny - 1), ny)
    iz = np.arange(-(nz - 1), nz)
    Z, Y, X = np.meshgrid(iz * d[2], iy * d[1], ix * d[0], indexing="ij")
    mult = ((nz - np.abs(iz))[:, None, None] * (ny - np.abs(iy))[None, :, None]
            * (nx - np.abs(ix))[None, None, :])
    a, b, c = nx * d[0] / 2, ny * d[1] / 2, nz * d[2] / 2
    ncell = nx * ny * nz
    nzz = np.sum(mult * newell_exact("zz", X, Y, Z, *d)) / ncell
    nxx = np.sum(mult * newell_exact("xx", X, Y, Z, *d)) / ncell
    nxy = np.sum(mult * newell_exact("xy", X, Y, Z, *d)) / ncell
    assert nzz == pytest.approx(aharoni_dz(a, b, c), rel=1e-11)
    assert nxx == pytest.approx(aharoni_dz(b, c, a), rel=1e-11)
    assert abs(nxy) < 1e-13


@pytest.mark.parametrize("comp", newell.COMPONENTS)
def test_far_field_approaches_dipole(comp):
    r = np.array([17.0, 9.0, -5.0])
    for scale in (1.0, 1.5):
        X, Y, Z = r * scale
        ex = newell_exact(comp, X, Y, Z, 1.0, 1.0, 1.0)
        dp = dipole(comp, X, Y, Z, 1.0, 1.0, 1.0)
        rr = np.linalg.norm(r * scale)
        # cubic cells: correction O((d/r)^4) relative to 1/(4 pi r^3)
        assert abs(ex - dp) * 4 * np.pi * rr ** 3 < 5.0 / rr ** 4 + 1e-6


def test_symmetries():
    X, Y, Z = 3.0, -2.0, 1.0
    c = (1.0, 1.0, 1.0)
    assert newell_exact("xx", -X, Y, Z, *c) == pytest.approx(newell_exact("xx", X, Y, Z, *c), rel=1e-12)
    assert newell_exact("xy", -X, Y, Z, *c) == pytest.approx(-newell_exact("xy", X, Y, Z, *c), rel=1e-12)
    assert newell_exact("xz", X, Y, -Z, *c) == pytest.approx(-newell_exact("xz", X, Y, Z, *c), rel=1e-12)
    assert newell_exact("yz", X, -Y, Z, *c) == pytest.approx(-newell_exact("yz", X, Y, Z, *c), rel=1e-12)
    # permutation consistency: N_yy(X,Y,Z) of a cube = N_xx(Y,X,Z)
    assert newell_exact("yy", X, Y, Z, *c) == pytest.approx(newell_exact("xx", Y, X, Z, *c), rel=1e-12)


def test_switch_radius_continuity():
    """At the switch radius the two definitions agree to ~1e-6 of the dipole scale."""
    for r in (30.0, 31.0):
        for comp in ("xx", "xy", "zz"):
            X, Y, Z = r * 0.6, r * 0.8, 0.0
            ex = newell_exact(comp, X, Y, Z, 1.0, 1.0, 1.0)
            dp = dipole(comp, X, Y, Z, 1.0, 1.0, 1.0)
            assert abs(ex - dp) * 4 * np.pi * r ** 3 < 3e-6


def test_float64_cancellation_bound_mpmath():
    """float64 Newell vs a 40-digit evaluation of the same difference."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40

    def f(x, y, z):
        x, y, z = abs(x), abs(y), abs(z)
        R = mp.sqrt(x * x + y * y + z * z)
        t = mp.mpf(0)
        if x * x + z * z > 0:
            t += y / 2 * (z * z - x * x) * mp.asinh(y / mp.sqrt(x * x + z * z))
        if x * x + y * y > 0:
            t += z / 2 * (y * y - x * x) * mp.asinh(z / mp.sqrt(x * x + y * y))
        if x * R > 0:
            t -= x * y * z * mp.atan(y * z / (x * R))
        return t + (2 * x * x - y * y - z * z) * R / 6

    W = {-1: -1, 0: 2, 1: -1}
    for (X, Y, Z) in ((5, 3, 1), (12, 7, 2), (20, 9, 4)):
        acc = mp.mpf(0)
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                for c in (-1, 0, 1):
                    acc += W[a] * W[b] * W[c] * f(mp.mpf(X + a), mp.mpf(Y + b), mp.mpf(Z + c))
        ref = float(acc / (4 * mp.pi))
        got = float(newell_exact("xx", float(X), float(Y), float(Z), 1.0, 1.0, 1.0))
        r = np.sqrt(X * X + Y * Y + Z * Z)
        assert abs(got - ref) * 4 * np.pi * r ** 3 < 1e-6
        # and the dipole limit is the physics it approaches
        assert abs(ref - float(dipole("xx", X, Y, Z, 1, 1, 1))) * 4 * np.pi * r ** 3 < 0.2


def test_demag_tensor_switch():
    X = np.array([0.0, 10.0, 40.0])
    out = demag_tensor("xx", X, 0.0, 0.0, 1.0, 1.0, 1.0, rc_cells=30.0)
    assert out[0] == pytest.approx(1 / 3)
    assert out[2] == dipole("xx", 40.0, 0.0, 0.0, 1, 1, 1)
