"""Eddy-current field of a conducting magnet (Sec. III.B, Eqs. 9-12).

Per time step, from the magnetisation at the start of the step:

1. B = mu0 (H_d + H_ext + Ms m) on the cells; dB/dt by the backward
   difference over the previous step, (B_n - B_{n-1}) / dt (the first step
   takes B_{-1} = B_0, i.e. no induced field before the first update).
2. Solenoidal field, Eq. (9): E_sol(r_i) = -sum_j dB_j/dt x S(r_i - r_j)
   = sum_j S(r_i - r_j) x dB_j/dt, with S the scalar-potential kernel of
   Eq. (8) (the integral of Eq. 10).  Eq. (11) as printed drops the minus
   sign of Eq. (9); the sign here is the one for which the discrete curl of
   E_sol is -dB/dt (Faraday), pinned in tests/test_oracle_eddy.py.
3. Irrotational field, Eq. (12): Laplace's equation for phi_E inside the
   magnet with d phi_E / dn = E_sol . n on its surface, E_irrot = -grad phi_E,
   so that J . n = 0.  Finite volumes on the cells: an interior face
   contributes (phi_j - phi_i) / d^2, a surface face s E_sol,a(i) / d with s
   the sign of its outward normal; the right-hand side is projected onto
   zero mean (compatibility of the pure Neumann problem) and phi has zero
   mean (gauge).  Solved by red-black successive over-relaxation (colour
   (i + j + k) mod 2, red first), omega = 2 / (1 + sin(pi / n_max)), a fixed
   number of sweeps per step from the previous step's phi.  A negative
   sweep count asks for the exact solution instead: the finite-volume
   Neumann Laplacian of a box is diagonal in the cosine basis
   cos(pi k (i + 1/2) / n) per axis (eigenvalue sum over axes of
   (2 cos(pi k / n) - 2) / d^2), so phi = DCT-III of (DCT-II of r / lambda)
   with the k = 0 mode (the gauge) set to zero.
   E_irrot,a(i) = -(g+ + g-) / 2 with g the face gradients, a surface face
   taking E_sol,a(i).
   A conductor periodic along an in-plane axis (pbc, the films of the
   friction geometry) has no surface across the period: its cells are
   neighbours through it, the Laplacian and the gradients wrap, and only
   the faces of the open axes carry E_sol . n.
4. J = sigma (E_sol + E_irrot) and H_eddy(r_i) = sum_j J_j x S(r_i - r_j)
   (Biot-Savart with the same kernel), held through the step's RK stages.

Pins (tests/test_oracle_eddy.py): the window sums equal brute-force sums;
the exact solve equals a sparse least-squares solve of the independently
assembled finite-volume system;
Faraday's law for a divergence-free dB/dt; the converged SOR equals a direct
sparse solve of the same system; a uniform E_sol is screened completely
(phi = E0 . r, so J = 0 in every cell and no current leaves the surface;
a flipped surface sign fails it); Lenz's law (the eddy field opposes a
growing uniform dB/dt).
"""
import numpy as np
from .constants import MU0
from .convolution import displacement_grid, WindowSum
from .potential_kernel import potential_kernel

EPS = {(0, 1, 2): 1.0, (1, 2, 0): 1.0, (2, 0, 1): 1.0,
       (0, 2, 1): -1.0, (2, 1, 0): -1.0, (1, 0, 2): -1.0}


def cross_kernels(desc, sign):
    """Kernels of out_a = sign * sum_c (S x v_c)_a, i.e. sign * eps_abc S_b v_c."""
    box = (0, desc.nx, 0, desc.ny, 0, desc.nz)
    X, Y, Z = displacement_grid(desc, box)
    S = potential_kernel(X, Y, Z, desc.dx, desc.dy, desc.dz)
    ker = {}
    for (a, b, c), e in EPS.items():
        ker[(a, c)] = ker.get((a, c), 0.0) + sign * e * S[b]
    return WindowSum(ker, (desc.nz, desc.ny, desc.nx), 3)


def periodic_axes(desc):
    """Array axes (of [nz][ny][nx]) along which the conductor is periodic:
    x (axis 2) for pbc bit 0, y (axis 1) for bit 1."""
    pbc = int(getattr(desc, "pbc", 0))
    return {ax for bit, ax in ((1, 2), (2, 1)) if pbc & bit}


def default_sweeps(desc):
    """Sweeps per step (0: 40); negative: the exact solve."""
    return desc.sor_sweeps if desc.sor_sweeps != 0 else 40


def neumann_solve(desc, r):
    """The zero-mean solution of L phi = r (L = laplacian below) for a
    zero-mean r, by the diagonalisation of L (module docstring): the cosine
    basis along an open axis, the Fourier basis exp(2 pi i k i / n),
    eigenvalue (2 cos(2 pi k / n) - 2) / d^2, along a periodic one."""
    from scipy.fft import dctn, idctn
    per = periodic_axes(desc)
    opn = tuple(a for a in range(3) if a not in per)
    nz, ny, nx = r.shape
    lam = np.zeros(r.shape)
    for axis, (n, d) in enumerate(((nz, desc.dz), (ny, desc.dy), (nx, desc.dx))):
        f = 2.0 if axis in per else 1.0
        ev = (2.0 * np.cos(f * np.pi * np.arange(n) / n) - 2.0) / (d * d)
        sh = [1, 1, 1]
        sh[axis] = n
        lam = lam + ev.reshape(sh)
    c = dctn(r, type=2, norm="ortho", axes=opn) if opn else np.array(r, dtype=np.float64)
    if per:
        c = np.fft.fftn(c, axes=tuple(sorted(per)))
    c[0, 0, 0] = 0.0
    lam[0, 0, 0] = 1.0
    c = c / lam
    if per:
        c = np.real(np.fft.ifftn(c, axes=tuple(sorted(per))))
    return idctn(c, type=2, norm="ortho", axes=opn) if opn else c


def default_omega(desc):
    if desc.sor_omega > 0:
        return desc.sor_omega
    n = max(desc.nx, desc.ny, desc.nz)
    return 2.0 / (1.0 + np.sin(np.pi / n))


def neumann_rhs(desc, Esol):
    """Right-hand side r of sum_interior (phi_j - phi_i)/d^2 = r_i."""
    r = np.zeros(Esol.shape[1:])
    per = periodic_axes(desc)
    for a, (axis, d) in enumerate(((2, desc.dx), (1, desc.dy), (0, desc.dz))):
        if axis in per:
            continue  # no surface across a period
        n = r.shape[axis]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, 1)
        hi[axis] = slice(n - 1, n)
        # + surface face: outward normal +a; - surface face: -a
        r[tuple(hi)] -= Esol[a][tuple(hi)] / d
        r[tuple(lo)] += Esol[a][tuple(lo)] / d
    return r - r.mean()


def laplacian(desc, phi):
    out = np.zeros_like(phi)
    per = periodic_axes(desc)
    for axis, d in ((2, desc.dx), (1, desc.dy), (0, desc.dz)):
        if axis in per:
            out += (np.roll(phi, 1, axis=axis) + np.roll(phi, -1, axis=axis) - 2.0 * phi) / (d * d)
            continue
        n = phi.shape[axis]
        if n < 2:
            continue
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        diff = (phi[tuple(hi)] - phi[tuple(lo)]) / (d * d)
        out[tuple(lo)] += diff
        out[tuple(hi)] -= diff
    return out


def neighbour_weight(desc, shape):
    """sum over interior faces of 1/d^2, per cell."""
    w = np.zeros(shape)
    per = periodic_axes(desc)
    for axis, d in ((2, desc.dx), (1, desc.dy), (0, desc.dz)):
        n = shape[axis]
        cnt = np.full(n, 2.0)
        if axis not in per:
            cnt[0] -= 1
            cnt[-1] -= 1
        sh = [1, 1, 1]
        sh[axis] = n
        w = w + cnt.reshape(sh) / (d * d)
    return w


def sor(desc, phi, r, sweeps, omega):
    """Red-black SOR sweeps (red = (i+j+k) even first), then zero mean."""
    nz, ny, nx = phi.shape
    for axis in periodic_axes(desc):
        assert phi.shape[axis] % 2 == 0, "red-black colouring needs even periods"
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    colour = (i + j + k) % 2
    W = neighbour_weight(desc, phi.shape)
    phi = phi.copy()
    for _ in range(sweeps):
        for c in (0, 1):
            # sum of neighbour values / d^2 over interior faces
            nb = laplacian(desc, phi) + W * phi
            upd = (nb - r) / W
            mask = colour == c
            phi[mask] = (1 - omega) * phi[mask] + omega * upd[mask]
    return phi - phi.mean()


def residual(desc, phi, r):
    """Relative L2 residual ||L phi - r|| / ||r|| of the Neumann problem
    (L = laplacian above), the measure of how far the fixed sweeps left phi
    from the solution."""
    res = laplacian(desc, phi) - r
    nr = float(np.sqrt((r * r).sum()))
    nres = float(np.sqrt((res * res).sum()))
    return nres / nr if nr > 0 else nres


def irrotational(desc, phi, Esol):
    """E_irrot = -(g+ + g-)/2 per axis; a surface face gradient is E_sol,a."""
    E = np.zeros_like(Esol)
    per = periodic_axes(desc)
    for a, (axis, d) in enumerate(((2, desc.dx), (1, desc.dy), (0, desc.dz))):
        n = phi.shape[axis]
        if axis in per:
            g = (np.roll(phi, -1, axis=axis) - phi) / d   # face i + 1/2, wrapping
            E[a] = -0.5 * (g + np.roll(g, 1, axis=axis))
            continue
        gp = np.array(Esol[a], copy=True)
        gm = np.array(Esol[a], copy=True)
        if n >= 2:
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[axis] = slice(0, n - 1)
            hi[axis] = slice(1, n)
            g = (phi[tuple(hi)] - phi[tuple(lo)]) / d
            gp[tuple(lo)] = g
            gm[tuple(hi)] = g
        E[a] = -0.5 * (gp + gm)
    return E


class EddyState:
    """Held eddy field and the history it needs (single conducting magnet)."""

    def __init__(self, desc):
        self.desc = desc
        shape = (3, desc.nz, desc.ny, desc.nx)
        self.H_eddy = np.zeros(shape)
        self.B_prev = None
        self.phi = np.zeros(shape[1:])
        self.r = np.zeros(shape[1:])
        self.E_sol = np.zeros(shape)
        self.J = np.zeros(shape)
        self._esol = None
        self._heddy = None

    def ops(self):
        if self._esol is None:
            self._esol = cross_kernels(self.desc, +1.0)   # E_sol = S x dB/dt
            self._heddy = cross_kernels(self.desc, -1.0)  # H = J x S = -S x J
        return self._esol, self._heddy

    def b_field(self, system, m):
        d = self.desc
        Hd = system.self_op()(m)
        h = np.asarray(d.Hext, dtype=np.float64)[:, None, None, None]
        return MU0 * (Hd + h + d.Ms * m)

    def update(self, system, dt):
        d = self.desc
        B = self.b_field(system, system.m[0])
        if self.B_prev is None:
            self.B_prev = B
        dB = (B - self.B_prev) / dt
        self.B_prev = B
        esol_op, heddy_op = self.ops()
        self.E_sol = esol_op(dB)
        r = neumann_rhs(d, self.E_sol)
        self.r = r
        sweeps = default_sweeps(d)
        self.phi = neumann_solve(d, r) if sweeps < 0 else sor(d, self.phi, r, sweeps, default_omega(d))
        self.J = d.sigma * (self.E_sol + irrotational(d, self.phi, self.E_sol))
        self.H_eddy = heddy_op(self.J)
