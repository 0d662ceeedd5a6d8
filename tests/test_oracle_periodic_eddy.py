"""Pins for eddy currents in films periodic in plane (Sec. III.B, Eqs. 9-12,
in the friction geometry of Sec. IV.B-C): the image-summed S x v window,
the periodic Neumann problem and the assembled update of two moving films."""
import numpy as np
import pytest
from workloads import Desc, Drive
from workloads.states import random_unit
from oracle.periodic import FilmSWindow, brute_force_s
from oracle.sim import FROZEN
from oracle.slab import SlabSystem, PeriodicLayers
from oracle import eddy as oracle_eddy


def film(pbc, nx=4, ny=4, nz=1, P=2, **kw):
    return Desc(n_films=2, nx=nx, ny=ny, nz=nz, dx=2e-9, dy=3e-9, dz=2.5e-9, Ms=9e5, pbc=pbc,
                pbc_images=P, halo=4, max_travel_cells=4, **kw)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("pbc", [1, 2, 3])
@pytest.mark.parametrize("box,dz", [((0, 4, 0, 4), 0), ((-2, 7, -1, 5), 2), ((3, 3, 2, 3), -3)])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_s_window_equals_brute_force_over_images(pbc, box, dz, sign):
    d = film(pbc)
    v = np.random.default_rng(pbc + 7 * abs(dz) + 3).standard_normal((3, 1, 4, 4))
    W = FilmSWindow(d, *box, dz, sign)(v)
    B = brute_force_s(d, v, *box, dz, sign)
    assert rel(W, B) < 1e-12


def assembled_solve(d, r):
    """The zero-mean least-squares solution of the finite-volume system
    assembled face by face: an interior face (or one through a period)
    between cells p and q adds (phi_q - phi_p) / h^2 to p's row."""
    from scipy.sparse import lil_matrix
    from scipy.sparse.linalg import lsqr
    nz, ny, nx = r.shape
    N = r.size
    A = lil_matrix((N, N))
    idx = lambda k, j, i: (k * ny + j) * nx + i
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = idx(k, j, i)
                for (dk, dj, di), h, n, per in (((0, 0, 1), d.dx, nx, d.pbc & 1), ((0, 1, 0), d.dy, ny, d.pbc & 2),
                                                ((1, 0, 0), d.dz, nz, 0)):
                    for s in (1, -1):
                        kk, jj, ii = k + s * dk, j + s * dj, i + s * di
                        c = (kk, jj, ii)[[dk, dj, di].index(1)]
                        if not 0 <= c < n:
                            if not per:
                                continue
                            kk, jj, ii = kk % nz, jj % ny, ii % nx
                        A[p, idx(kk, jj, ii)] += 1.0 / h ** 2
                        A[p, p] -= 1.0 / h ** 2
    phi = lsqr(A.tocsr(), r.ravel(), atol=1e-15, btol=1e-15, iter_lim=20000)[0].reshape(r.shape)
    return phi - phi.mean()


@pytest.mark.parametrize("pbc", [1, 2, 3])
def test_periodic_neumann_solves_equal_the_assembled_system(pbc):
    d = film(pbc, nx=6, ny=4, nz=3)
    rng = np.random.default_rng(pbc)
    r = rng.standard_normal((3, 4, 6))
    r -= r.mean()
    ref = assembled_solve(d, r)
    exact = oracle_eddy.neumann_solve(d, r)
    assert rel(exact, ref) < 1e-9
    sor = oracle_eddy.sor(d, np.zeros_like(r), r, 400, oracle_eddy.default_omega(d))
    assert rel(sor, ref) < 1e-8
    assert oracle_eddy.residual(d, exact, r) < 1e-12


@pytest.mark.parametrize("pbc", [0, 1, 2, 3])
def test_uniform_field_drives_current_only_along_the_periods(pbc):
    """A uniform E_sol is screened along the open axes (the surface charge
    cancels it inside) and drives sigma E along the periodic ones, where no
    surface closes the current."""
    d = film(pbc, nx=6, ny=4, nz=3, sigma=2e6)
    E0 = np.array([1.5, -0.7, 0.9])
    Es = np.tile(E0[:, None, None, None], (1, 3, 4, 6))
    r = oracle_eddy.neumann_rhs(d, Es)
    for phi in (oracle_eddy.neumann_solve(d, r),
                oracle_eddy.sor(d, np.zeros_like(r), r, 600, oracle_eddy.default_omega(d))):
        J = d.sigma * (Es + oracle_eddy.irrotational(d, phi, Es))
        want = d.sigma * E0 * np.array([pbc & 1 != 0, pbc & 2 != 0, False])
        assert np.abs(J - want[:, None, None, None]).max() < 1e-7 * d.sigma * np.abs(E0).max()


def test_uniform_perpendicular_rate_has_no_solenoidal_field_in_a_periodic_film():
    """E_sol = S x dB/dt of a uniform dB/dt along z: in a film periodic in x
    and y every source has its mirror image, and the odd in-plane components
    of S cancel; an open film has a circulating E_sol."""
    rate = np.tile(np.array([0.0, 0.0, 1.0])[:, None, None, None], (1, 2, 4, 6))
    d = film(3, nx=6, ny=4, nz=2)
    E = PeriodicLayers(d, (0, 6, 0, 4, 0, 2), +1.0)(rate)
    Eo = oracle_eddy.cross_kernels(d.replace(pbc=0), +1.0)(rate)
    assert np.abs(Eo).max() > 0
    assert np.abs(E).max() < 1e-12 * np.abs(Eo).max()


@pytest.mark.parametrize("pbc,axis,shift", [(1, 3, 2), (2, 2, 1), (3, 3, 5)])
def test_periodic_eddy_update_commutes_with_a_translation(pbc, axis, shift):
    """Rolling both films' magnetisation and dB/dt along a periodic axis rolls
    every eddy quantity the update assembles (E_sol, phi, J, H_eddy of both
    films, own and cross sums): nothing of an open boundary is left along it.
    At an integer offset, where the interpolant returns the window's values
    (at a fractional one the mirrored ends of the 4-cell halo move with the
    data)."""
    d = film(pbc, nx=6, ny=4, nz=2, sigma=1e6, sor_sweeps=-1, gap_cells=1)
    rng = np.random.default_rng(11 * pbc)
    m = [random_unit((2, 4, 6), rng) for _ in range(2)]
    rate = [1e10 * rng.standard_normal((3, 2, 4, 6)) for _ in range(2)]
    dt = 1e-13
    out = []
    for k in (0, shift):
        mk = [np.roll(a, k, axis=axis) for a in m]
        s = SlabSystem(d, Drive(mode=FROZEN, x0=2.0 * d.dx), mk)
        B = s.eddy.b_fields(s)
        s.eddy.B_prev = [B[f] - dt * np.roll(rate[f], k, axis=axis) for f in range(2)]
        s.eddy.update(s, dt)
        out.append(s.eddy)
    for f in range(2):
        for name in ("E_sol", "J", "H"):
            a = np.roll(getattr(out[0], name)[f], shift, axis=axis)
            b = getattr(out[1], name)[f]
            assert rel(b, a) < 1e-9, (f, name)
        assert rel(out[1].phi[f], np.roll(out[0].phi[f], shift, axis=axis - 1)) < 1e-9


def test_periodic_gradient_is_the_central_difference_of_a_sampled_wave():
    """E_irrot along a periodic axis is minus the mean of the two face
    gradients, i.e. minus the central difference: for phi = cos(2 pi q i / n)
    that is sin(2 pi q / n) / d * sin(2 pi q i / n) (a trigonometric
    identity), whatever E_sol holds."""
    d = film(1, nx=8, ny=4, nz=2)
    q = 3
    i = np.arange(8)
    phi = np.tile(np.cos(2 * np.pi * q * i / 8), (2, 4, 1))
    Es = np.random.default_rng(4).standard_normal((3, 2, 4, 8))
    E = oracle_eddy.irrotational(d, phi, Es)
    want = np.sin(2 * np.pi * q / 8) / d.dx * np.sin(2 * np.pi * q * i / 8)
    assert np.abs(E[0] - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("pbc", [1, 3])
def test_sor_sweeps_are_the_red_black_sor_of_the_assembled_matrix(pbc):
    """A fixed number of sweeps (as the step runs them) equals the textbook
    SOR update phi_p <- (1 - w) phi_p + w (r_p - sum_q!=p A_pq phi_q) / A_pp on
    the assembled matrix, red cells ((i + j + k) even) first, then the zero
    mean."""
    from scipy.sparse import lil_matrix
    d = film(pbc, nx=6, ny=4, nz=3)
    rng = np.random.default_rng(3 + pbc)
    r = rng.standard_normal((3, 4, 6))
    r -= r.mean()
    phi0 = rng.standard_normal((3, 4, 6))
    omega, sweeps = 1.37, 3
    got = oracle_eddy.sor(d, phi0, r, sweeps, omega)
    nz, ny, nx = r.shape
    A = lil_matrix((r.size, r.size))
    idx = lambda k, j, i: (k * ny + j) * nx + i
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = idx(k, j, i)
                for (dk, dj, di), h, n, per in (((0, 0, 1), d.dx, nx, d.pbc & 1), ((0, 1, 0), d.dy, ny, d.pbc & 2),
                                                ((1, 0, 0), d.dz, nz, 0)):
                    for s in (1, -1):
                        kk, jj, ii = k + s * dk, j + s * dj, i + s * di
                        c = (kk, jj, ii)[[dk, dj, di].index(1)]
                        if not 0 <= c < n and not per:
                            continue
                        A[p, idx(kk % nz, jj % ny, ii % nx)] += 1.0 / h ** 2
                        A[p, p] -= 1.0 / h ** 2
    A = A.toarray()
    x = phi0.ravel().copy()
    rv = r.ravel()
    colour = np.array([(k + j + i) % 2 for k in range(nz) for j in range(ny) for i in range(nx)])
    for _ in range(sweeps):
        for c in (0, 1):
            new = x.copy()
            for p in np.nonzero(colour == c)[0]:
                off = A[p] @ x - A[p, p] * x[p]
                new[p] = (1 - omega) * x[p] + omega * (rv[p] - off) / A[p, p]
            x = new
    want = (x - x.mean()).reshape(r.shape)
    assert rel(got, want) < 1e-12
