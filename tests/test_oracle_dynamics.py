"""Pins for the LLG integrator, the energy balance of Eq. (4) and the slider EOM."""
import math
import numpy as np
import pytest
from workloads import Desc, Drive
from workloads.states import random_unit, domain_state
from oracle.constants import GAMMA0
from oracle.sim import System, SPRING, FROZEN


def macrospin(alpha, H, theta0, phi0, dt, n):
    d = Desc(n_films=1, nx=1, ny=1, nz=1, dx=3e-9, dy=3e-9, dz=3e-9, Ms=8e5,
             Aex=1e-11, alpha=alpha, Hext=(0.0, 0.0, H))
    m = np.zeros((3, 1, 1, 1))
    m[:, 0, 0, 0] = [math.sin(theta0) * math.cos(phi0),
                     math.sin(theta0) * math.sin(phi0), math.cos(theta0)]
    s = System(d, Drive(), [m])
    s.run(dt, n)
    mm = s.m[0][:, 0, 0, 0]
    return s.t, mm


def test_macrospin_closed_form():
    alpha, H, th0, ph0 = 0.1, 1e5, 0.5, 0.2
    t, mm = macrospin(alpha, H, th0, ph0, 1e-13, 2000)
    g = GAMMA0 / (1 + alpha ** 2)
    th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * g * H * t))
    ph = ph0 + g * H * t
    ref = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    assert np.abs(mm - ref).max() < 1e-9


def two_film(nx=12, ny=10, gap=1, xp=0.0, alpha=0.5, seed=0, mode=FROZEN, **kw):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=5e-9, dy=5e-9, dz=5e-9,
             gap_cells=gap, Ms=8e5, Aex=1.3e-11, alpha=alpha, Ku=0.0, **kw)
    rng = np.random.default_rng(seed)
    m = [random_unit((1, ny, nx), rng) for _ in range(2)]
    return System(d, Drive(mode=mode, x0=xp * d.dx), m)


def test_energy_decay_equals_dissipation():
    """Eq. (4): with the slider at a lattice position dE/dt = -P_diss."""
    s = two_film(xp=0.0)
    dt = 2e-15
    E0 = s.energies()["total"]
    P0 = s.p_diss()
    s.step(dt)
    E1 = s.energies()["total"]
    P1 = s.p_diss()
    dEdt = (E1 - E0) / dt
    assert dEdt < 0
    assert dEdt == pytest.approx(-0.5 * (P0 + P1), rel=1e-4)


def test_unit_norm_and_rk4_order():
    errs = []
    ref = two_film(xp=0.37, seed=1)
    ref.run(2.5e-14, 16)
    for n, dt in ((4, 1e-13), (8, 5e-14)):
        s = two_film(xp=0.37, seed=1)
        s.run(dt, n)
        assert np.allclose(np.sum(s.m[1] ** 2, axis=0), 1.0, atol=1e-14)
        errs.append(max(np.abs(a - b).max() for a, b in zip(s.m, ref.m)))
    # fourth order: halving dt cuts the error ~16x (renormalisation aside)
    assert errs[0] / errs[1] > 10


class NoCross(System):
    def cross_fields(self, m_b, m_s, x, s_int, want_force=True):
        z = np.zeros_like(m_b)
        return z, z, np.zeros(3)


def test_spring_slider_critical_damping():
    d = Desc(n_films=2, nx=4, ny=4, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, Ms=1e6, alpha=0.1)
    k, M = 1e-3, 1e-20
    w0 = math.sqrt(k / M)
    drv = Drive(mode=SPRING, v_d=1.0, k=k, mass=M, gamma_v=2 * w0)
    rng = np.random.default_rng(0)
    s = NoCross(d, drv, [random_unit((1, 4, 4), rng) for _ in range(2)])
    dt = 2e-11
    s.run(dt, 100)
    t = s.t
    vd = 1.0
    x_ref = vd * t - 2 * vd / w0 + (2 * vd / w0 + vd * t) * math.exp(-w0 * t)
    assert s.x == pytest.approx(x_ref, rel=1e-9)
    assert s.s_int == math.floor(s.x / d.dx)


def test_force_symmetry_and_sign():
    d = Desc(n_films=2, nx=12, ny=9, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, Ms=1e6, gap_cells=1)
    m = np.zeros((3, 1, 9, 12))
    m[2] = 1.0
    s = System(d, Drive(mode=FROZEN, x0=0.0), [m, m.copy()])
    F = s.force()
    assert abs(F[0]) < 1e-12 * abs(F[2]) and abs(F[1]) < 1e-12 * abs(F[2])
    assert F[2] < 0   # stacked parallel perpendicular films attract
    s.x = 0.3 * d.dx
    F = s.force()
    assert F[0] < 0   # restoring towards alignment
    # base/slider field relation for identical uniform films (x-mirror + z-mirror)
    for xp in (0.0, 0.3):
        Hb, Hs, _ = s.cross_fields(m, m, xp * d.dx, 0)
        sc = np.abs(Hs).max()
        assert np.abs(Hb[2, 0] - Hs[2, 0][:, ::-1]).max() < 1e-11 * sc
        assert np.abs(Hb[0, 0] - Hs[0, 0][:, ::-1]).max() < 1e-11 * sc
        assert np.abs(Hb[1, 0] + Hs[1, 0][:, ::-1]).max() < 1e-11 * sc


def test_force_is_minus_energy_gradient():
    # Eq. (3) with two-point differences vs the derivative of the interpolated
    # energy: equal up to the O(d^2) difference error (1-4% for smooth domain
    # states, larger for cell-scale random states).
    d = Desc(n_films=2, nx=48, ny=40, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, Ms=1.1e6, gap_cells=3)
    m = [domain_state((1, 40, 48), 11), domain_state((1, 40, 48), 12)]
    s = System(d, Drive(mode=FROZEN), m)
    x = 0.4 * d.dx
    h = 0.02 * d.dx
    e = lambda xx: s.energies(x=xx)["demag_cross"]
    dEdx = (e(x + h) - e(x - h)) / (2 * h)
    s.x = x
    F = s.force()
    assert F[0] == pytest.approx(-dEdx, rel=3e-2)


def test_reseat_continuity():
    """Crossing a cell boundary only moves the window's mirror ends."""
    s = two_film(nx=40, ny=6, xp=0.0, seed=4)
    m_b, m_s = s.m
    Hb0, Hs0, _ = s.cross_fields(m_b, m_s, 1.0 * s.desc.dx, 0)
    Hb1, Hs1, _ = s.cross_fields(m_b, m_s, 1.0 * s.desc.dx, 1)
    sl = slice(12, 28)
    scale = np.abs(Hs0).max()
    assert np.abs(Hs0[..., sl] - Hs1[..., sl]).max() < 1e-7 * scale
    assert np.abs(Hs0 - Hs1).max() < 5e-2 * scale


@pytest.mark.parametrize("gap,kind,tol", [(3, "dom", 1e-2), (5, "rand", 1e-2)])
def test_potential_mode_matches_direct_far_field(gap, kind, tol):
    # Point-sampled -grad(phi) vs the cell-averaged tensor field: both are the
    # same harmonic field away from the source, up to discretisation error.
    d = Desc(n_films=2, nx=48, ny=40, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, Ms=1.1e6,
             gap_cells=gap)
    if kind == "dom":
        m = [domain_state((1, 40, 48), 11), domain_state((1, 40, 48), 12)]
    else:
        rng = np.random.default_rng(0)
        m = [random_unit((1, 40, 48), rng) for _ in range(2)]
    x = 0.4 * d.dx
    sd = System(d, Drive(mode=FROZEN, x0=x), m)
    sp = System(d.replace(cross_mode=1), Drive(mode=FROZEN, x0=x), m)
    Hbd, Hsd, Fd = sd.cross_fields(*m, x, 0)
    Hbp, Hsp, Fp = sp.cross_fields(*m, x, 0)
    inner = (slice(None), slice(None), slice(3, -3), slice(3, -3))
    assert np.abs(Hsd - Hsp)[inner].max() < tol * np.abs(Hsd).max()
    assert np.abs(Hbd - Hbp)[inner].max() < tol * np.abs(Hbd).max()
    assert Fp[0] == pytest.approx(Fd[0], rel=tol)
