"""Pins for the eddy-current field (Sec. III.B, Eqs. 9-12)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from workloads import Desc, Drive
from oracle import eddy
from oracle.convolution import direct_sum
from oracle.potential_kernel import potential_kernel


def cube(n, d=1e-9, **kw):
    return Desc(n_films=1, nx=n[0], ny=n[1], nz=n[2], dx=d, dy=d, dz=d, Ms=8e5, sigma=1e7, **kw)


def test_cross_sums_equal_brute_force():
    d = cube((3, 4, 2))
    rng = np.random.default_rng(1)
    v = rng.standard_normal((3, 2, 4, 3))

    def kfn(X, Y, Z):
        S = potential_kernel(X, Y, Z, d.dx, d.dy, d.dz)
        K = np.zeros((3, 3) + S.shape[1:])
        for (a, b, c), e in eddy.EPS.items():
            K[a, c] += e * S[b]
        return K

    ref = direct_sum(kfn, d, v, (0, 3, 0, 4, 0, 2))
    got = eddy.cross_kernels(d, +1.0)(v)
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert np.allclose(eddy.cross_kernels(d, -1.0)(v), -ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def bump_field(n, d, sigma=4.5):
    """dB/dt = curl (0, 0, psi) for a Gaussian bump psi: divergence-free."""
    c = (np.array(n) - 1) / 2.0
    k, j, i = np.meshgrid(*(np.arange(m) for m in n[::-1]), indexing="ij")
    x, y = (i - c[0]) * d, (j - c[1]) * d
    z = (k - c[2]) * d
    s = sigma * d
    psi = np.exp(-(x * x + y * y + z * z) / (2 * s * s))
    B = np.zeros((3,) + psi.shape)
    B[0] = -y / (s * s) * psi       # d psi / dy
    B[1] = x / (s * s) * psi        # -d psi / dx
    return B


def curl(E, d):
    g = [np.gradient(E[a], d, axis=(2, 1, 0)) for a in range(3)]  # g[a][0]=d/dx ...
    return np.array([g[2][1] - g[1][2], g[0][2] - g[2][0], g[1][0] - g[0][1]])


def test_faraday_sign():
    n = (30, 30, 30)
    d = cube(n)
    Bdot = bump_field(n, d.dx)
    E = eddy.cross_kernels(d, +1.0)(Bdot)
    c = curl(E, d.dx)
    inner = (slice(None), slice(8, -8), slice(8, -8), slice(8, -8))
    err = np.abs(c + Bdot)[inner].max() / np.abs(Bdot).max()
    assert err < 0.05            # curl E_sol = -dB/dt up to discretisation
    err_wrong = np.abs(c - Bdot)[inner].max() / np.abs(Bdot).max()
    assert err_wrong > 1.5       # the sign printed in Eq. (11) would fail


def fv_matrix(d, shape):
    nz, ny, nx = shape
    idx = np.arange(nx * ny * nz).reshape(shape)
    rows, cols, vals = [], [], []
    for axis, h in ((2, d.dx), (1, d.dy), (0, d.dz)):
        n = shape[axis]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        a, b = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        w = 1.0 / (h * h)
        rows += [a, b, a, b]
        cols += [b, a, a, b]
        vals += [np.full(a.size, w), np.full(a.size, w), np.full(a.size, -w), np.full(a.size, -w)]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(idx.size, idx.size))
    return A


def test_sor_converges_to_direct_solve():
    shape = (5, 6, 8)
    d = cube(shape[::-1], d=2e-9)
    rng = np.random.default_rng(3)
    Esol = rng.standard_normal((3,) + shape)
    r = eddy.neumann_rhs(d, Esol)
    assert abs(r.sum()) < 1e-12 * np.abs(r).sum()
    A = fv_matrix(d, shape)
    # pure Neumann: append the zero-mean gauge as an extra row
    N = r.size
    Aa = sp.vstack([A, sp.csr_matrix(np.ones((1, N)))])
    sol = spla.lsqr(Aa, np.concatenate([r.ravel(), [0.0]]), atol=1e-15, btol=1e-15, iter_lim=20000)[0]
    phi = eddy.sor(d, np.zeros(shape), r, 3000, eddy.default_omega(d))
    assert np.abs(phi.ravel() - sol).max() < 1e-10 * np.abs(sol).max()
    assert np.abs(eddy.laplacian(d, phi) - r).max() < 1e-9 * np.abs(r).max()


def test_residual_against_the_sparse_matrix():
    """eddy.residual is ||A phi - r|| / ||r|| with A the finite-volume
    matrix assembled independently (fv_matrix): checked on a random phi, on
    phi = 0 (residual 1) and on the converged solve (tiny); more sweeps leave
    a smaller residual."""
    shape = (4, 5, 7)
    d = cube(shape[::-1], d=2e-9)
    rng = np.random.default_rng(8)
    r = eddy.neumann_rhs(d, rng.standard_normal((3,) + shape))
    A = fv_matrix(d, shape)
    phi = rng.standard_normal(shape)
    ref = np.linalg.norm(A @ phi.ravel() - r.ravel()) / np.linalg.norm(r)
    assert eddy.residual(d, phi, r) == pytest.approx(ref, rel=1e-12)
    assert eddy.residual(d, np.zeros(shape), r) == pytest.approx(1.0, rel=1e-14)
    om = eddy.default_omega(d)
    res = [eddy.residual(d, eddy.sor(d, np.zeros(shape), r, n, om), r) for n in (1, 10, 40, 2000)]
    assert res[0] > res[1] > res[2] > res[3] and res[3] < 1e-9


def test_lenz_law():
    n = (12, 12, 12)
    d = cube(n, d=2e-9)
    Bdot = np.zeros((3, 12, 12, 12))
    Bdot[2] = 1e9                        # uniform growing B along z (T/s)
    st = eddy.EddyState(d)
    esol, heddy = st.ops()
    E = esol(Bdot)
    r = eddy.neumann_rhs(d, E)
    phi = eddy.sor(d, np.zeros(n[::-1]), r, 400, eddy.default_omega(d))
    J = d.sigma * (E + eddy.irrotational(d, phi, E))
    H = heddy(J)
    assert H[2, 6, 6, 6] < 0 and H[2, 5, 5, 5] < 0
    # currents circulate about z, clockwise seen from +z for a growing B_z
    assert J[1, 6, 6, 10] < 0 < J[1, 6, 6, 1]
    assert J[0, 6, 10, 6] > 0 > J[0, 6, 1, 6]


def test_update_history_and_units():
    from oracle.sim import System
    n = (6, 5, 4)
    d = cube(n, d=2e-9).replace(Hext=(0.0, 0.0, -3e4), sor_sweeps=5)
    m = np.zeros((3, 4, 5, 6))
    m[2] = 1.0
    s = System(d, Drive(), [m])
    s.step(1e-14)
    # first step: dB/dt taken as zero -> no induced field yet
    assert np.abs(s.eddy.H_eddy).max() == 0.0
    s.step(1e-14)
    assert np.abs(s.eddy.H_eddy).max() > 0.0


def _uniform_field_current(d, shape, E0, rhs=eddy.neumann_rhs):
    Esol = np.zeros((3,) + shape)
    for a in range(3):
        Esol[a] = E0[a]
    r = rhs(d, Esol)
    phi = eddy.sor(d, np.zeros(shape), r, 3000, eddy.default_omega(d))
    return d.sigma * (Esol + eddy.irrotational(d, phi, Esol)), d.sigma * np.linalg.norm(E0)


def test_uniform_field_is_screened_no_current_leaves():
    # A uniform solenoidal field inside an insulated conductor is cancelled
    # by the surface charge: phi = E0 . r solves Laplace's equation with
    # d phi / dn = E0 . n on every face, so E_irrot = -E0 and J = 0 in every
    # cell, in particular no current crosses the surface (Eq. 12).
    shape = (5, 6, 7)
    d = cube(shape[::-1], d=2e-9)
    J, scale = _uniform_field_current(d, shape, np.array([3.0, -2.0, 1.5]))
    assert np.abs(J).max() < 1e-9 * scale


def test_uniform_field_pin_rejects_flipped_surface_sign():
    shape = (5, 6, 7)
    d = cube(shape[::-1], d=2e-9)
    J, scale = _uniform_field_current(d, shape, np.array([3.0, -2.0, 1.5]),
                                      rhs=lambda dd, E: -eddy.neumann_rhs(dd, E))
    assert np.abs(J).max() > 0.5 * scale


@pytest.mark.parametrize("shape", [(5, 6, 8), (2, 7, 3), (1, 4, 9)])
def test_exact_neumann_solve_equals_the_sparse_solve(shape):
    """The cosine-basis solve (sor_sweeps < 0) against a least-squares solve
    of the independently assembled finite-volume system with the zero-mean
    gauge row; anisotropic cells; one-cell-thin axes included."""
    d = cube(shape[::-1], d=2e-9).replace(dy=3e-9, dz=1.5e-9, sor_sweeps=-1)
    rng = np.random.default_rng(sum(shape))
    r = eddy.neumann_rhs(d, rng.standard_normal((3,) + shape))
    A = fv_matrix(d, shape)
    N = r.size
    Aa = sp.vstack([A, sp.csr_matrix(np.ones((1, N)))])
    sol = spla.lsqr(Aa, np.concatenate([r.ravel(), [0.0]]), atol=1e-15, btol=1e-15, iter_lim=50000)[0]
    phi = eddy.neumann_solve(d, r)
    assert abs(phi.sum()) < 1e-12 * np.abs(phi).sum()
    assert np.abs(phi.ravel() - sol).max() < 1e-9 * np.abs(sol).max()
    assert eddy.residual(d, phi, r) < 1e-12
