"""Two thick films in relative motion, with eddy currents in both
(Sec. II.A end, Sec. III.B, Eqs. 9-12; Sec. IV.C, IV.D).

TEST INFRASTRUCTURE ONLY (part of the float64 oracle).

Geometry.  As in oracle.sim, but each film is nx x ny x nz cells (nz >= 1)
and the slider's lattice origin sits z_s = nz + gap layers above the base's.
Every cross mode: the direct field with the cubic B-spline along x
(cross_mode 0) or linear interpolation (2), and the scalar potential (1).
Open in-plane boundaries, or periodic ones (pbc, every cross mode): every
layer pair's sum then takes oracle.periodic's image-summed kernel (the
potential's too), window points outside the period take their image's
value (for the potential, the copy of Sec. III.A end), and exchange wraps
(the paper's friction films, Sec. IV.B; its eddy-current friction run,
Sec. IV.C, keeps that geometry).  With eddy currents the eddy sums take the
image-summed S kernel the same way and each film's Neumann problem is
periodic along those axes (oracle.eddy).

Cross fields.  The base's exact lattice field is computed on the slider's
window of base-lattice points x in [s_int - h, s_int + nx + h), rows
[-1, ny] and layers z_s - 1 .. z_s + nz (the slider's layers and one more
on each side for the force), prefiltered along x and sampled at
x = i + s_int + x_p.  The slider's field is computed on the base's window
(x in [-s_int - h, -s_int + nx + h), rows [0, ny), layers -z_s .. -z_s + nz
- 1 of the slider's lattice, i.e. the base's layers) and sampled at
x = i - s_int - x_p.  With nz = 1 these are the windows of oracle.sim.

Scalar-potential mode (Sec. II.A, III.A, Eqs. 7-8).  The base's potential is
computed on the slider's window with rows [-3, ny + 2] and layers z_s - 3 ..
z_s + nz + 2, the slider's on the base's window with rows [-2, ny + 1] and
layers -z_s - 2 .. -z_s + nz + 1; each window row is prefiltered along x and
sampled at the shifted lattice, and H = -grad phi by the four-point central
difference along every axis (as oracle.sim, layer by layer).

Force (Eq. 3).  F = mu0 Ms V sum over every slider cell of (m . grad) H
with two-point central differences of the interpolated base field; the
z neighbours of the slider's bottom and top layers are the window layers
z_s - 1 and z_s + nz.

Eddy currents in both films (readings, listed in the design notes):
* each film is its own conductor: B = mu0 (H_d + H_ext + Ms m) on its cells,
  H_d the film's own field plus the other film's interpolated field, and
  dB/dt is the backward difference of B over the last step at the film's
  own cells (so it contains the change the motion causes; first step zero);
* the solenoidal field of Eq. 9 on a film sums the dB/dt of both films:
  its own cells by the lattice sum of oracle.eddy, the other film's cells
  on the window above, sampled at the film's shifted cells with the cross
  field's interpolant (an induced field is not a gradient, so its vectors
  are interpolated directly, Sec. II.A);
* one Neumann problem per film (Eq. 12; the currents cannot cross the gap),
  the finite-volume system and red-black SOR of oracle.eddy;
* the Biot-Savart field of the currents J = sigma (E_sol + E_irrot) sums
  both films the same way; the eddy field of a film is its own currents'
  field plus the other film's, interpolated (Sec. IV.C, IV.D);
* the eddy fields are computed from the state at the start of a step and
  held through its RK stages (as in oracle.eddy); Eq. 3's force is the
  base's stray field only.

Non-uniform applied field (Sec. II.A; the reading of oracle.applied, layer
by layer): film 0 takes its values on its cells, (3, nz, ny, nx); the
slider's layers take the frame field (3, nz, ny, nx + 2 (max_travel_cells +
halo)) sampled at their moved cells with the cross field's interpolant.  It
enters the Zeeman term, and so B of the eddy update; not the force.

Pins (tests/test_oracle_slab.py): at integer offsets the thick-film cross
fields, the force and the cross eddy sums equal brute-force sums over
physical cell centres; nz = 1 reproduces oracle.sim's fields at a
fractional offset; films far apart reduce each film's eddy field to the
single-magnet eddy field of oracle.eddy.
"""
import numpy as np

from .constants import MU0
from .convolution import displacement_grid, WindowSum
from .potential_kernel import potential_kernel
from .spline import prefilter, interp_1d, linear_1d
from .sim import System
from .applied import slider_width
from . import eddy as _eddy


def s_cross_window(desc, box, sign):
    """out_a(p) = sign * sum_j (S(p - r_j) x v_j)_a on `box` (Eq. 9 and the
    Biot-Savart sum of the currents, with the kernel S of Eq. 8)."""
    X, Y, Z = displacement_grid(desc, box)
    S = potential_kernel(X, Y, Z, desc.dx, desc.dy, desc.dz)
    ker = {}
    for (a, b, c), e in _eddy.EPS.items():
        ker[(a, c)] = ker.get((a, c), 0.0) + sign * e * S[b]
    return WindowSum(ker, (desc.nz, desc.ny, desc.nx), 3)


class SlabSystem(System):
    """Oracle state and fields of two films nz >= 1 cells thick."""

    def __init__(self, desc, drive=None, m_init=None):
        assert desc.n_films == 2, "two films"
        # the base class would set up the single-magnet eddy state
        super().__init__(desc.replace(sigma=0.0), drive, m_init)
        self.desc = desc
        self.eddy = FilmEddy(desc) if desc.sigma > 0 else None
        # non-uniform applied field of each film (module docstring); None = none
        self.hext_thick = [None, None]

    # ------------------------------------------------------------ windows
    def self_op(self):
        d = self.desc
        if d.pbc:
            return self._op(("self",), lambda: PeriodicLayers(d, (0, d.nx, 0, d.ny, 0, d.nz)))
        return super().self_op()

    def cross_op(self, direction, s_int):
        d = self.desc
        if d.pbc:
            box = self.cross_box(direction, s_int)
            pot = d.cross_mode == 1
            return self._op(("cross", direction, s_int, d.cross_mode),
                            lambda: PeriodicLayers(d, box, potential=pot))
        return super().cross_op(direction, s_int)

    def cross_box(self, direction, s_int):
        d = self.desc
        h, zs, nwx = d.halo, d.z_s, d.nx + 2 * d.halo
        if d.cross_mode == 1:
            if direction == "b2s":
                return (s_int - h, nwx, -3, d.ny + 6, zs - 3, d.nz + 6)
            return (-s_int - h, nwx, -2, d.ny + 4, -zs - 2, d.nz + 4)
        if direction == "b2s":
            return (s_int - h, nwx, -1, d.ny + 2, zs - 1, d.nz + 2)
        return (-s_int - h, nwx, 0, d.ny, -zs, d.nz)

    @staticmethod
    def grad4(c, t0, r0, u, n_l, ny, steps):
        """-grad phi by four-point central differences at window layers t0 ..
        t0 + n_l - 1, rows r0 .. r0 + ny - 1 and positions u, from the
        prefiltered potential window c (layers, rows, M): (3, n_l, ny, nx)."""
        def p(t, r, uu):
            return np.stack([interp_1d(c[t + k, r:r + ny], uu) for k in range(n_l)])

        def d4(fm2, fm1, fp1, fp2, hh):
            return (fm2 - 8.0 * fm1 + 8.0 * fp1 - fp2) / (12.0 * hh)

        dx, dy, dz = steps
        hx = -d4(p(t0, r0, u - 2), p(t0, r0, u - 1), p(t0, r0, u + 1), p(t0, r0, u + 2), dx)
        hy = -d4(p(t0, r0 - 2, u), p(t0, r0 - 1, u), p(t0, r0 + 1, u), p(t0, r0 + 2, u), dy)
        hz = -d4(p(t0 - 2, r0, u), p(t0 - 1, r0, u), p(t0 + 1, r0, u), p(t0 + 2, r0, u), dz)
        return np.array([hx, hy, hz])

    def interpolant(self):
        """The interpolant of field vectors along x (direct cross field, eddy
        sums, applied field): linear in cross_mode 2, else the spline."""
        if self.desc.cross_mode == 2:
            return (lambda G: G), linear_1d
        return (lambda G: prefilter(G, axis=-1)), interp_1d

    def positions(self, x, s_int, direction):
        """Window coordinates of the target film's cells along x."""
        d = self.desc
        xp = x / d.dx - s_int
        ii = np.arange(d.nx, dtype=np.float64) + d.halo
        return ii + xp if direction == "b2s" else ii - xp

    # --------------------------------------------------------- cross field
    def base_field_stencil(self, m_b, x, s_int):
        """The base's field at the slider's cells ("c") and at their six
        neighbour points, each (3, nz, ny, nx) [A/m]."""
        d = self.desc
        ny, nz = d.ny, d.nz
        u = self.positions(x, s_int, "b2s")
        if d.cross_mode == 1:
            # potential window: slider layer l at window layer l + 3, row j at j + 3
            cphi = prefilter(self.cross_op("b2s", s_int)(m_b)[0], axis=-1)
            st = (d.dx, d.dy, d.dz)
            g = self.grad4
            return {"c": g(cphi, 3, 3, u, nz, ny, st),
                    "xp": g(cphi, 3, 3, u + 1, nz, ny, st), "xm": g(cphi, 3, 3, u - 1, nz, ny, st),
                    "yp": g(cphi, 3, 4, u, nz, ny, st), "ym": g(cphi, 3, 2, u, nz, ny, st),
                    "zp": g(cphi, 4, 3, u, nz, ny, st), "zm": g(cphi, 2, 3, u, nz, ny, st)}
        pre, samp = self.interpolant()
        c = pre(self.cross_op("b2s", s_int)(m_b))     # (3, nz+2, ny+2, M)
        L, R = slice(1, nz + 1), slice(1, ny + 1)
        return {"c": samp(c[:, L, R], u),
                "xp": samp(c[:, L, R], u + 1), "xm": samp(c[:, L, R], u - 1),
                "yp": samp(c[:, L, 2:ny + 2], u), "ym": samp(c[:, L, 0:ny], u),
                "zp": samp(c[:, 2:nz + 2, R], u), "zm": samp(c[:, 0:nz, R], u)}

    def cross_fields(self, m_b, m_s, x, s_int, want_force=True):
        """(H on base, H on slider, F[3]); fields (3, nz, ny, nx)."""
        d = self.desc
        pre, samp = self.interpolant()
        st = self.base_field_stencil(m_b, x, s_int)
        F = np.zeros(3)
        if want_force:
            V = d.dx * d.dy * d.dz
            dHdx = (st["xp"] - st["xm"]) / (2 * d.dx)
            dHdy = (st["yp"] - st["ym"]) / (2 * d.dy)
            dHdz = (st["zp"] - st["zm"]) / (2 * d.dz)
            F = MU0 * d.Ms * V * (m_s[0][None] * dHdx + m_s[1][None] * dHdy
                                  + m_s[2][None] * dHdz).sum(axis=(1, 2, 3))
        if d.cross_mode == 1:
            # base layer k at window layer k + 2, row j at j + 2
            cb = prefilter(self.cross_op("s2b", s_int)(m_s)[0], axis=-1)
            Hb = self.grad4(cb, 2, 2, self.positions(x, s_int, "s2b"), d.nz, d.ny, (d.dx, d.dy, d.dz))
            return Hb, st["c"], F
        Gb = pre(self.cross_op("s2b", s_int)(m_s))     # (3, nz, ny, M)
        Hb = samp(Gb, self.positions(x, s_int, "s2b"))
        return Hb, st["c"], F

    def slider_hext(self, x, s_int):
        """The slider's non-uniform applied field at its cells, (3, nz, ny, nx)."""
        d = self.desc
        hs = np.asarray(self.hext_thick[1], dtype=np.float64)
        assert hs.shape == (3, d.nz, d.ny, slider_width(d)), hs.shape
        cols = s_int - d.halo + np.arange(d.nx + 2 * d.halo)
        if d.pbc & 1:
            cols = np.mod(cols, d.nx)
        else:
            cols = cols + d.max_travel_cells + d.halo
            assert cols.min() >= 0 and cols.max() < hs.shape[-1], "slider beyond the applied field's columns"
        pre, samp = self.interpolant()
        return samp(pre(hs[..., cols]), self.positions(x, s_int, "b2s"))

    def field_terms(self, m_list=None, x=None, s_int=None, want_force=True):
        out, F = super().field_terms(m_list, x, s_int, want_force)
        x = self.x if x is None else x
        s_int = self.s_int if s_int is None else s_int
        if self.hext_thick[0] is not None:
            out[0]["zeeman"] = out[0]["zeeman"] + np.asarray(self.hext_thick[0], dtype=np.float64)
        if self.hext_thick[1] is not None:
            out[1]["zeeman"] = out[1]["zeeman"] + self.slider_hext(x, s_int)
        if self.eddy is not None:
            for f in range(2):
                out[f]["eddy"] = self.eddy.H[f].copy()
        return out, F


class PeriodicLayers:
    """The stray field of a thick film with periodic in-plane axes on a box
    of target points (x0, nwx, y0, nwy, z0, nwz): target layer z0 + k takes
    the sum over source layers l of oracle.periodic.FilmWindow at the layer
    offset z0 + k - l; output (3, nwz, nwy, nwx) like WindowSum.  With a
    sign, the eddy-current sum sign * S x v instead (FilmSWindow); with
    potential, the scalar potential (one channel, FilmPotWindow)."""

    def __init__(self, desc, box, sign=None, potential=False):
        from .periodic import FilmWindow, FilmSWindow, FilmPotWindow
        x0, nwx, y0, nwy, z0, nwz = box
        self.nwz, self.z0, self.nz = nwz, z0, desc.nz

        def window(dz):
            if potential:
                return FilmPotWindow(desc, x0, nwx, y0, nwy, dz)
            if sign is None:
                return FilmWindow(desc, x0, nwx, y0, nwy, dz)
            return FilmSWindow(desc, x0, nwx, y0, nwy, dz, sign)
        self.win = {dz: window(dz) for dz in range(z0 - (desc.nz - 1), z0 + nwz)}

    def __call__(self, m):
        out = None
        for k in range(self.nwz):
            layer = sum(self.win[self.z0 + k - l](m[:, l:l + 1]) for l in range(self.nz))
            out = layer if out is None else np.concatenate([out, layer], axis=1)
        return out


class FilmEddy:
    """Eddy-current state of both films (module docstring)."""

    def __init__(self, desc):
        d = desc
        assert d.nz >= 2 and d.ny >= 2 and d.nx >= 2, \
            "eddy currents need films more than one cell thick in every direction"
        shape = (3, d.nz, d.ny, d.nx)
        self.desc = d
        self.H = [np.zeros(shape), np.zeros(shape)]
        self.E_sol = [np.zeros(shape), np.zeros(shape)]
        self.J = [np.zeros(shape), np.zeros(shape)]
        self.phi = [np.zeros(shape[1:]), np.zeros(shape[1:])]
        self.r = [np.zeros(shape[1:]), np.zeros(shape[1:])]
        self.B_prev = [None, None]
        self._self = None
        self._cross = {}

    @property
    def H_eddy(self):
        """The base film's eddy field (the single-magnet state's name)."""
        return self.H[0]

    def self_ops(self):
        d = self.desc
        if self._self is None and d.pbc:
            box = (0, d.nx, 0, d.ny, 0, d.nz)
            self._self = (PeriodicLayers(d, box, +1.0), PeriodicLayers(d, box, -1.0))
        if self._self is None:
            self._self = (_eddy.cross_kernels(d, +1.0), _eddy.cross_kernels(d, -1.0))
        return self._self

    def cross_box(self, direction, s_int):
        d = self.desc
        h, zs, nwx = d.halo, d.z_s, d.nx + 2 * d.halo
        if direction == "b2s":
            return (s_int - h, nwx, 0, d.ny, zs, d.nz)
        return (-s_int - h, nwx, 0, d.ny, -zs, d.nz)

    def cross_op(self, sign, direction, s_int):
        key = (sign, direction, s_int)
        if key not in self._cross and self.desc.pbc:
            self._cross[key] = PeriodicLayers(self.desc, self.cross_box(direction, s_int), sign)
        if key not in self._cross:
            self._cross[key] = s_cross_window(self.desc, self.cross_box(direction, s_int), sign)
        return self._cross[key]

    def cross_sum(self, system, sign, direction, src, x, s_int):
        """sign * sum over the source film's cells of S x src, sampled at the
        target film's cells: direction "b2s" sources the base and targets the
        slider, "s2b" the reverse."""
        pre, samp = system.interpolant()
        G = pre(self.cross_op(sign, direction, s_int)(src))
        return samp(G, system.positions(x, s_int, direction))

    def b_fields(self, system):
        d = self.desc
        terms, _ = system.field_terms(want_force=False)
        return [MU0 * (t["demag_self"] + t["demag_cross"] + t["zeeman"] + d.Ms * m)
                for t, m in zip(terms, system.m)]

    def update(self, system, dt):
        d = self.desc
        x, s_int = system.x, system.s_int
        B = self.b_fields(system)
        dB = []
        for f in range(2):
            if self.B_prev[f] is None:
                self.B_prev[f] = B[f]
            dB.append((B[f] - self.B_prev[f]) / dt)
            self.B_prev[f] = B[f]
        esol, hop = self.self_ops()
        self.E_sol = [esol(dB[0]) + self.cross_sum(system, +1.0, "s2b", dB[1], x, s_int),
                      esol(dB[1]) + self.cross_sum(system, +1.0, "b2s", dB[0], x, s_int)]
        sweeps, omega = _eddy.default_sweeps(d), _eddy.default_omega(d)
        for f in range(2):
            self.r[f] = _eddy.neumann_rhs(d, self.E_sol[f])
            self.phi[f] = (_eddy.neumann_solve(d, self.r[f]) if sweeps < 0
                           else _eddy.sor(d, self.phi[f], self.r[f], sweeps, omega))
            self.J[f] = d.sigma * (self.E_sol[f] + _eddy.irrotational(d, self.phi[f], self.E_sol[f]))
        self.H = [hop(self.J[0]) + self.cross_sum(system, -1.0, "s2b", self.J[1], x, s_int),
                  hop(self.J[1]) + self.cross_sum(system, -1.0, "b2s", self.J[0], x, s_int)]
