"""Pins for the thick two-film oracle with eddy currents (oracle.slab;
Sec. II.A, III.A-B, Eqs. 3, 6, 9-12; Sec. IV.C-D).

At an integer offset (x_p = 0) the spline reproduces the window data
exactly, so every sampled field, the force of Eq. 3 and the cross-film
eddy sums must equal brute-force sums over source cells written here from
the physical cell centres alone: base cell (i, j, l) at ((i+1/2) dx,
(j+1/2) dy, (l+1/2) dz), slider cell at (x_s + (i+1/2) dx, (j+1/2) dy,
(z_s + l + 1/2) dz) with z_s = nz + gap.  Nothing below reuses the
oracle's window boxes, its FFT sums or its stencil helper.  Two reductions
pin the rest: one-cell-thick films reproduce oracle.sim at a fractional
offset, and films far apart reduce each film's eddy field to the
single-magnet field of oracle.eddy.
"""
import numpy as np
import pytest
from workloads import Desc, Drive
from workloads.states import random_unit
from oracle.constants import MU0
from oracle.newell import tensor_matrix
from oracle.potential_kernel import potential_kernel
from oracle.sim import System, FROZEN
from oracle.slab import SlabSystem
from oracle import eddy as oracle_eddy

EPS = {(0, 1, 2): 1.0, (1, 2, 0): 1.0, (2, 0, 1): 1.0,
       (0, 2, 1): -1.0, (2, 1, 0): -1.0, (1, 0, 2): -1.0}


def films(nx=6, ny=4, nz=2, gap=1, seed=5, **kw):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=nz, dx=2e-9, dy=3e-9, dz=2.5e-9,
             gap_cells=gap, Ms=9e5, halo=4, max_travel_cells=4, **kw)
    rng = np.random.default_rng(seed)
    m = [random_unit((nz, ny, nx), rng) for _ in range(2)]
    return d, m


def centres(d, x_shift, z0):
    """Cell centres of a film whose lowest layer has index z0, (nz, ny, nx)."""
    kk, jj, ii = np.meshgrid(np.arange(d.nz), np.arange(d.ny), np.arange(d.nx), indexing="ij")
    return (ii + 0.5) * d.dx + x_shift, (jj + 0.5) * d.dy, (kk + z0 + 0.5) * d.dz


def tensor_field_at(d, P, src, x_shift, z0):
    X, Y, Z = centres(d, x_shift, z0)
    N = tensor_matrix(P[0] - X, P[1] - Y, P[2] - Z, d.dx, d.dy, d.dz, d.rc_cells)
    return np.array([-d.Ms * sum(np.sum(N[a, b] * src[b]) for b in range(3)) for a in range(3)])


def s_cross_at(d, P, v, x_shift, z0):
    """sum_j (S(P - r_j) x v_j) over a film's cells."""
    X, Y, Z = centres(d, x_shift, z0)
    S = potential_kernel(P[0] - X, P[1] - Y, P[2] - Z, d.dx, d.dy, d.dz)
    out = np.zeros(3)
    for (a, b, c), e in EPS.items():
        out[a] += e * np.sum(S[b] * v[c])
    return out


def brute_force(d, m, s_int):
    mb, ms = m
    zs = d.nz + d.gap_cells
    xs = s_int * d.dx
    steps = np.array([d.dx, d.dy, d.dz])
    shape = (3, d.nz, d.ny, d.nx)
    Hs, Hb, F = np.zeros(shape), np.zeros(shape), np.zeros(3)
    V = d.dx * d.dy * d.dz
    for k in range(d.nz):
        for j in range(d.ny):
            for i in range(d.nx):
                Ps = np.array([xs + (i + 0.5) * d.dx, (j + 0.5) * d.dy, (zs + k + 0.5) * d.dz])
                Pb = np.array([(i + 0.5) * d.dx, (j + 0.5) * d.dy, (k + 0.5) * d.dz])
                Hs[:, k, j, i] = tensor_field_at(d, Ps, mb, 0.0, 0)
                Hb[:, k, j, i] = tensor_field_at(d, Pb, ms, xs, zs)
                for a in range(3):
                    e = np.zeros(3)
                    e[a] = steps[a]
                    dH = (tensor_field_at(d, Ps + e, mb, 0.0, 0)
                          - tensor_field_at(d, Ps - e, mb, 0.0, 0)) / (2 * steps[a])
                    F += MU0 * d.Ms * V * ms[a, k, j, i] * dH
    return Hb, Hs, F


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("nz,s_int,gap", [(2, 0, 1), (2, 3, 2), (3, -2, 1)])
def test_thick_cross_fields_and_force_equal_brute_force(nz, s_int, gap):
    d, m = films(nz=nz, gap=gap, seed=nz + 7 * abs(s_int))
    sysm = SlabSystem(d, Drive(mode=FROZEN, x0=s_int * d.dx), m)
    Hb, Hs, F = sysm.cross_fields(m[0], m[1], s_int * d.dx, s_int)
    rb, rs, rF = brute_force(d, m, s_int)
    assert Hb.shape == Hs.shape == (3, nz, d.ny, d.nx)
    assert rel(Hs, rs) < 1e-10
    assert rel(Hb, rb) < 1e-10
    assert np.abs(F - rF).max() < 1e-9 * np.abs(rF).max()


def test_linear_mode_equals_spline_mode_at_integer_offsets():
    d, m = films(nz=2)
    a = SlabSystem(d, Drive(mode=FROZEN, x0=2 * d.dx), m).cross_fields(m[0], m[1], 2 * d.dx, 2)
    b = SlabSystem(d.replace(cross_mode=2), Drive(mode=FROZEN, x0=2 * d.dx), m).cross_fields(
        m[0], m[1], 2 * d.dx, 2)
    for u, v in zip(a, b):
        assert rel(u, v) < 1e-11


@pytest.mark.parametrize("cross_mode", [0, 2])
def test_one_layer_reduces_to_the_film_oracle(cross_mode):
    d, m = films(nx=9, ny=5, nz=1, cross_mode=cross_mode)
    x = 1.37 * d.dx
    a = SlabSystem(d, Drive(mode=FROZEN, x0=x), m).cross_fields(m[0], m[1], x, 1)
    b = System(d, Drive(mode=FROZEN, x0=x), m).cross_fields(m[0], m[1], x, 1)
    for u, v in zip(a, b):
        assert rel(u, v) < 1e-12


@pytest.mark.parametrize("direction,s_int", [("b2s", 0), ("b2s", 2), ("s2b", -1)])
def test_cross_eddy_sums_equal_brute_force(direction, s_int):
    d, _ = films(nz=2, gap=2, sigma=1e6)
    sysm = SlabSystem(d, Drive(mode=FROZEN, x0=s_int * d.dx),
                      [np.tile(np.array([0, 0, 1.0])[:, None, None, None], (1, 2, d.ny, d.nx))] * 2)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((3, d.nz, d.ny, d.nx))
    zs = d.nz + d.gap_cells
    xs = s_int * d.dx
    for sign in (+1.0, -1.0):
        got = sysm.eddy.cross_sum(sysm, sign, direction, v, xs, s_int)
        ref = np.zeros_like(got)
        for k in range(d.nz):
            for j in range(d.ny):
                for i in range(d.nx):
                    if direction == "b2s":   # base sources, slider cells
                        P = np.array([xs + (i + 0.5) * d.dx, (j + 0.5) * d.dy, (zs + k + 0.5) * d.dz])
                        ref[:, k, j, i] = sign * s_cross_at(d, P, v, 0.0, 0)
                    else:                    # slider sources, base cells
                        P = np.array([(i + 0.5) * d.dx, (j + 0.5) * d.dy, (k + 0.5) * d.dz])
                        ref[:, k, j, i] = sign * s_cross_at(d, P, v, xs, zs)
        assert rel(got, ref) < 1e-10


def test_far_films_reduce_to_the_single_magnet_eddy_field():
    d, m = films(nx=5, ny=4, nz=3, gap=400, sigma=2e6, seed=11)
    d = d.replace(sor_sweeps=30)
    dt = 1e-13
    rng = np.random.default_rng(4)
    m2 = [mm + 0.05 * rng.standard_normal(mm.shape) for mm in m]
    m2 = [mm / np.linalg.norm(mm, axis=0, keepdims=True) for mm in m2]
    slab = SlabSystem(d, Drive(mode=FROZEN), m)
    singles = [System(d.replace(n_films=1, gap_cells=0), Drive(), [m[f]]) for f in range(2)]
    for state in (m, m2):
        slab.m = [s.copy() for s in state]
        slab.eddy.update(slab, dt)
        for f in range(2):
            singles[f].m = [state[f].copy()]
            singles[f].eddy.update(singles[f], dt)
    for f in range(2):
        ref = singles[f].eddy.H_eddy
        assert np.abs(ref).max() > 0
        assert rel(slab.eddy.H[f], ref) < 1e-5


def test_moving_films_with_eddy_currents_step():
    """Two RK4 steps with eddy currents and a moving slider stay finite and
    normalised; the held eddy fields change with the motion."""
    d, m = films(nx=6, ny=4, nz=2, gap=1, sigma=1e6, seed=2)
    drv = Drive(mode=1, v_d=50.0, x0=0.4 * d.dx)
    s = SlabSystem(d, drv, m)
    s.run(2e-13, 3)
    for f in range(2):
        assert np.all(np.isfinite(s.eddy.H[f]))
        assert np.abs(s.eddy.H[f]).max() > 0
        assert np.allclose(np.linalg.norm(s.m[f], axis=0), 1.0, atol=1e-12)
    assert s.x > 0.4 * d.dx


def test_eddy_update_sums_both_films_with_the_right_signs():
    """E_sol and H_eddy of each film, assembled by the update at an integer
    offset, equal brute-force sums over both films' cells: E = sum S x dB/dt,
    H = -sum S x J (Eq. 9 and the Biot-Savart field of the currents)."""
    d, m = films(nx=5, ny=3, nz=2, gap=1, sigma=1e6, seed=8)
    s_int, dt = 1, 1e-13
    slab = SlabSystem(d, Drive(mode=FROZEN, x0=s_int * d.dx), m)
    rng = np.random.default_rng(9)
    # about 1e-3 T per step: the backward difference keeps ~13 digits
    rate = [1e10 * rng.standard_normal((3, d.nz, d.ny, d.nx)) for _ in range(2)]
    B = slab.eddy.b_fields(slab)
    slab.eddy.B_prev = [B[f] - dt * rate[f] for f in range(2)]
    slab.eddy.update(slab, dt)
    zs = d.nz + d.gap_cells
    xs = s_int * d.dx
    origin = [(0.0, 0), (xs, zs)]
    for f in range(2):
        E = np.zeros((3, d.nz, d.ny, d.nx))
        H = np.zeros_like(E)
        for k in range(d.nz):
            for j in range(d.ny):
                for i in range(d.nx):
                    P = np.array([origin[f][0] + (i + 0.5) * d.dx, (j + 0.5) * d.dy,
                                  (origin[f][1] + k + 0.5) * d.dz])
                    for g in range(2):
                        E[:, k, j, i] += s_cross_at(d, P, rate[g], *origin[g])
                        H[:, k, j, i] -= s_cross_at(d, P, slab.eddy.J[g], *origin[g])
        assert rel(slab.eddy.E_sol[f], E) < 1e-10
        assert rel(slab.eddy.H[f], H) < 1e-10


@pytest.mark.parametrize("cross_mode", [0, 2])
def test_thick_applied_field_is_the_film_sampling_layer_by_layer(cross_mode):
    """The slider's applied field in thick films equals oracle.applied's
    (pinned) sampling of each layer; a uniform field is exact."""
    from oracle.applied import slider_samples, slider_width
    d, m = films(nx=9, ny=5, nz=3, cross_mode=cross_mode)
    rng = np.random.default_rng(12)
    hs = rng.standard_normal((3, d.nz, d.ny, slider_width(d)))
    s = SlabSystem(d, Drive(mode=FROZEN), m)
    s.hext_thick = [None, hs]
    d1 = d.replace(nz=1)
    for x_cells in (0.0, 1.37, -2.5, 4.0):
        s_int = int(np.floor(x_cells))
        got = s.slider_hext(x_cells * d.dx, s_int)
        for layer in range(d.nz):
            ref = slider_samples(d1, hs[:, layer], x_cells * d.dx, s_int)
            assert np.allclose(got[:, layer], ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    s.hext_thick = [None, np.broadcast_to(np.array([1.0, -2.0, 3.0])[:, None, None, None], hs.shape)]
    got = s.slider_hext(1.37 * d.dx, 1)
    assert np.allclose(got, np.array([1.0, -2.0, 3.0])[:, None, None, None], rtol=0, atol=1e-12)


def test_thick_films_energy_decays_with_a_frozen_slider():
    """With the slider held still, no eddy currents and strong damping, the
    total energy (exchange, anisotropy, Zeeman, own and cross stray fields)
    decreases step by step: the thick-film fields are the gradient of the
    energy the integrator dissipates."""
    d, m = films(nx=8, ny=6, nz=3, gap=1, seed=4, alpha=0.8, Ku=2e5, Hext=(1e4, 0.0, 2e4))
    s = SlabSystem(d, Drive(mode=FROZEN, x0=1.4 * d.dx), m)
    e = [s.energies()["total"]]
    for _ in range(12):
        s.step(2e-13)
        e.append(s.energies()["total"])
    assert all(b < a for a, b in zip(e, e[1:])), e


def potential_at(d, P, src, x_shift, z0):
    """phi(P) = Ms sum_j S(P - r_j) . m_j over a film's cells."""
    X, Y, Z = centres(d, x_shift, z0)
    S = potential_kernel(P[0] - X, P[1] - Y, P[2] - Z, d.dx, d.dy, d.dz)
    return d.Ms * sum(np.sum(S[b] * src[b]) for b in range(3))


def grad4_at(fun, P, steps):
    H = np.zeros(3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = steps[a]
        H[a] = -(fun(P - 2 * e) - 8 * fun(P - e) + 8 * fun(P + e) - fun(P + 2 * e)) / (12 * steps[a])
    return H


@pytest.mark.parametrize("nz,s_int", [(2, 0), (3, 2)])
def test_thick_potential_mode_equals_brute_force(nz, s_int):
    """Scalar-potential mode at integer offsets: the four-point differences of
    a brute-force potential at the cell centres, and Eq. 3's force from them."""
    d, m = films(nx=6, ny=5, nz=nz, gap=3, seed=nz + 3 * s_int, cross_mode=1)
    sysm = SlabSystem(d, Drive(mode=FROZEN, x0=s_int * d.dx), m)
    Hb, Hs, F = sysm.cross_fields(m[0], m[1], s_int * d.dx, s_int)
    zs = d.nz + d.gap_cells
    xs = s_int * d.dx
    steps = np.array([d.dx, d.dy, d.dz])
    rb, rs, rF = np.zeros_like(Hb), np.zeros_like(Hs), np.zeros(3)
    V = d.dx * d.dy * d.dz

    def base_field(P):
        return grad4_at(lambda Q: potential_at(d, Q, m[0], 0.0, 0), P, steps)

    for k in range(d.nz):
        for j in range(d.ny):
            for i in range(d.nx):
                Ps = np.array([xs + (i + 0.5) * d.dx, (j + 0.5) * d.dy, (zs + k + 0.5) * d.dz])
                Pb = np.array([(i + 0.5) * d.dx, (j + 0.5) * d.dy, (k + 0.5) * d.dz])
                rs[:, k, j, i] = base_field(Ps)
                rb[:, k, j, i] = grad4_at(lambda Q: potential_at(d, Q, m[1], xs, zs), Pb, steps)
                for a in range(3):
                    e = np.zeros(3)
                    e[a] = steps[a]
                    rF += MU0 * d.Ms * V * m[1][a, k, j, i] * (base_field(Ps + e) - base_field(Ps - e)) / (2 * steps[a])
    assert rel(Hs, rs) < 1e-9
    assert rel(Hb, rb) < 1e-9
    assert np.abs(F - rF).max() < 1e-8 * np.abs(rF).max()


def test_thick_potential_mode_one_layer_reduces_to_the_film_oracle():
    d, m = films(nx=9, ny=5, nz=1, gap=3, cross_mode=1)
    x = 1.37 * d.dx
    a = SlabSystem(d, Drive(mode=FROZEN, x0=x), m).cross_fields(m[0], m[1], x, 1)
    b = System(d, Drive(mode=FROZEN, x0=x), m).cross_fields(m[0], m[1], x, 1)
    for u, v in zip(a, b):
        assert rel(u, v) < 1e-12


@pytest.mark.parametrize("pbc", [1, 2, 3])
def test_periodic_thick_films_one_layer_reduces_to_the_film_oracle(pbc):
    """Periodic thick films with nz = 1 are the pinned periodic film oracle."""
    d, m = films(nx=8, ny=6, nz=1, gap=1, seed=pbc)
    d = d.replace(pbc=pbc, pbc_images=2)
    x = 1.37 * d.dx
    a = SlabSystem(d, Drive(mode=FROZEN, x0=x), m)
    b = System(d, Drive(mode=FROZEN, x0=x), m)
    ta, Fa = a.field_terms()
    tb, Fb = b.field_terms()
    for f in range(2):
        for k in ("exchange", "demag_self", "demag_cross"):
            assert rel(ta[f][k], tb[f][k]) < 1e-12, (f, k)
    assert np.abs(Fa - Fb).max() <= 1e-12 * np.abs(Fb).max()


def test_periodic_thick_films_physics():
    """A uniform magnetisation gives the same field in every cell of a layer
    (translation invariance along both periodic axes); shifting the slider by
    one period leaves every field and the force unchanged; with many images a
    uniformly perpendicular periodic film tends to H_z = -Ms in its middle."""
    d, m = films(nx=8, ny=6, nz=3, gap=1, seed=6)
    d = d.replace(pbc=3, pbc_images=2, max_travel_cells=16)
    up = [np.tile(np.array([0.1, -0.2, 0.97])[:, None, None, None], (1, 3, 6, 8))] * 2
    s = SlabSystem(d, Drive(mode=FROZEN, x0=1.3 * d.dx), up)
    t, _ = s.field_terms()
    for f in range(2):
        for k in ("demag_self", "demag_cross"):
            h = t[f][k]
            assert np.abs(h - h[:, :, :1, :1]).max() < 1e-9 * np.abs(h).max(), (f, k)
    s1 = SlabSystem(d, Drive(mode=FROZEN, x0=1.3 * d.dx), m)
    s2 = SlabSystem(d, Drive(mode=FROZEN, x0=(1.3 + d.nx) * d.dx), m)
    t1, F1 = s1.field_terms()
    t2, F2 = s2.field_terms()
    for f in range(2):
        assert rel(t2[f]["demag_cross"], t1[f]["demag_cross"]) < 1e-12
    assert np.abs(F2 - F1).max() <= 1e-12 * np.abs(F1).max()
    dz = d.replace(nx=6, ny=6, nz=1, pbc_images=60, dx=2e-9, dy=2e-9, dz=2e-9)
    zup = [np.tile(np.array([0.0, 0.0, 1.0])[:, None, None, None], (1, 1, 6, 6))] * 2
    hz = SlabSystem(dz, Drive(mode=FROZEN), zup).field_terms()[0][0]["demag_self"][2]
    assert abs(hz.mean() / dz.Ms + 1.0) < 0.02
