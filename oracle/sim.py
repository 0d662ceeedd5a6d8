"""Two magnets, one fixed (base, film 0) and one moving (slider, film 1).

Geometry (Sec. II, Fig. 3; Sec. III).  Each film is its own finite-
difference lattice of nx x ny x 1 cells.  The base's lattice origin is 0;
the slider sits z_s = nz + gap layers higher and is displaced along x by
x_s = (s_int + x_p) dx, s_int = floor(x_s / dx) held fixed within a time
step and updated after it (the paper's full-cell re-seat, Sec. III).  The
films interact only through the stray field (Sec. II.A, Eq. 2).

Cross fields, direct mode (Sec. II.A, III.A).  The exact lattice field of
the base, G(p) = -Ms sum_j N(p - r_j) m_j, is computed on the slider's
window of base-lattice points x in [s_int - h, s_int + nx + h), rows
[-1, ny] and layers z_s-1..z_s+1; it is prefiltered along x
(oracle.spline) and sampled at x = i + s_int + x_p.  The base samples the
slider's field the same way at x = i - s_int - x_p.

Cross fields, scalar-potential mode (Sec. II.A, III.A, Eqs. 7-8).  The
potential phi(p) = Ms sum_j S(p - r_j).m_j is computed on the window,
spline-sampled on the shifted lattice and differentiated with the
four-point central difference (f(-2) - 8 f(-1) + 8 f(+1) - f(+2)) / (12 d).
Only the far field is taken from the potential: points within one cell of
the source magnet's box would take the tensor value, which for films at
least one empty layer apart never happens to a slider cell.

Force (Sec. III, Eq. 3).  F = mu0 Ms V sum_{i in slider} (m_i . grad) H,
grad the two-point central difference of the interpolated base field at
the neighbouring points of the shifted lattice.

Time stepping (Sec. III; Eq. 15).  Classic RK4 on (m_base, m_slider, x_s,
v_s); every stage evaluates H_eff at its own (m, x_s, t); m is
renormalised after the step.  Drives: frozen, constant velocity, or
m x'' = k (v_d t + x_a0 - x) - gamma_v m x' + F_x.

Parity: at integer offsets the cross fields of both films and the force
of Eq. 3 equal brute-force sums over physical cell centres, in direct mode
(tensor) and potential mode (four-point differences of the brute-force
potential), which pins the window layers, rows, offset signs and the
stencil (tests/test_oracle_cross.py, with planted slips rejected); the
spline's sub-cell sampling is pinned by its own tests; F_x = 0 for
mirror-symmetric states, F_x ~ -dE_cross/dx_s and base/slider reaction;
energy decay pins the integrator.
"""
import math
import numpy as np
from .constants import MU0, GAMMA0
from . import fields as _fields
from .llg import llg_rhs
from .convolution import demag_window, potential_window
from .spline import prefilter, interp_1d, linear_1d

FROZEN, VELOCITY, SPRING = 0, 1, 2
TERMS = ("exchange", "anisotropy", "zeeman", "demag_self", "demag_cross",
         "eddy")


def _d4(fm2, fm1, fp1, fp2, h):
    return (fm2 - 8.0 * fm1 + 8.0 * fp1 - fp2) / (12.0 * h)


class System:
    """Oracle state and fields for one problem (see module docstring)."""

    def __init__(self, desc, drive=None, m_init=None):
        from workloads.desc import Drive
        self.desc = desc
        self.drive = drive if drive is not None else Drive()
        self.m = [np.array(m, dtype=np.float64) for m in m_init]
        assert len(self.m) == desc.n_films
        self.t = 0.0
        self.x = float(self.drive.x0)
        self.v = float(self.drive.v0)
        if self.drive.mode == VELOCITY:
            self.v = self.drive.v_d
        self.s_int = int(math.floor(self.x / desc.dx))
        self.step_count = 0
        self._ops = {}
        self.eddy = None
        # optional replacement of the base film's cross field: a callable
        # (m_slider, x_s) -> H [A/m] (used to compose with the learned operator)
        self.base_cross = None
        # non-uniform applied field (oracle/applied.py): film 0 on its cells,
        # the slider's layer on the frame lattice; None = uniform Hext only
        self.hext_fields = [None, None]
        if desc.sigma > 0:
            from .eddy import EddyState
            self.eddy = EddyState(desc)

    # ------------------------------------------------------------ windows
    def _op(self, key, maker):
        if key not in self._ops:
            self._ops[key] = maker()
        return self._ops[key]

    def self_op(self):
        d = self.desc
        if d.pbc:
            from .periodic import BoxWindow
            assert d.nz == 1, "periodic boundaries: films one cell thick"
            return self._op(("self",), lambda: BoxWindow(d, (0, d.nx, 0, d.ny, 0, 1)))
        return self._op(("self",), lambda: demag_window(
            d, (0, d.nx, 0, d.ny, 0, d.nz)))

    def cross_box(self, direction, s_int):
        """Target box (x0, nwx, y0, nwy, z0, nwz) in the source film's lattice."""
        d = self.desc
        h, zs = d.halo, d.z_s
        nwx = d.nx + 2 * h
        if d.cross_mode in (0, 2):
            if direction == "b2s":
                return (s_int - h, nwx, -1, d.ny + 2, zs - 1, 3)
            return (-s_int - h, nwx, 0, d.ny, -zs, 1)
        if direction == "b2s":
            return (s_int - h, nwx, -3, d.ny + 6, zs - 3, 7)
        return (-s_int - h, nwx, -2, d.ny + 4, -zs - 2, 5)

    def cross_op(self, direction, s_int):
        d = self.desc
        box = self.cross_box(direction, s_int)
        if d.pbc:
            # periodic films: the window is the periodic field (or potential),
            # its halo the copy from the other side
            from .periodic import BoxWindow
            return self._op(("cross", direction, s_int, d.cross_mode),
                            lambda: BoxWindow(d, box, potential=d.cross_mode == 1))
        maker = (lambda: demag_window(d, box)) if d.cross_mode in (0, 2) else (
            lambda: potential_window(d, box))
        return self._op(("cross", direction, s_int, d.cross_mode), maker)

    # --------------------------------------------------------- cross field
    def cross_fields(self, m_b, m_s, x, s_int, want_force=True):
        """Interpolated stray fields and the force on the slider.

        Returns (H_on_base, H_on_slider, F[3]); H arrays have shape
        (3, 1, ny, nx).
        """
        d = self.desc
        h = d.halo
        xp = x / d.dx - s_int
        ii = np.arange(d.nx, dtype=np.float64)
        u_s = ii + h + xp        # slider cells in the base-field window
        u_b = ii + h - xp        # base cells in the slider-field window
        V = d.dx * d.dy * d.dz
        ny = d.ny
        F = np.zeros(3)
        if d.cross_mode in (0, 2):
            # cubic B-spline (mode 0) or linear interpolation (mode 2) of the
            # window data along the motion axis
            pre = prefilter if d.cross_mode == 0 else (lambda G, axis: G)
            samp = interp_1d if d.cross_mode == 0 else linear_1d
            st = self.base_field_stencil(m_b, x, s_int)
            Hs = st["c"]
            if want_force:
                ms = m_s[:, 0]
                dHdx = (st["xp"] - st["xm"]) / (2 * d.dx)
                dHdy = (st["yp"] - st["ym"]) / (2 * d.dy)
                dHdz = (st["zp"] - st["zm"]) / (2 * d.dz)
                F = MU0 * d.Ms * V * (ms[0][None] * dHdx + ms[1][None] * dHdy
                                      + ms[2][None] * dHdz).sum(axis=(1, 2))
            Gb = self.cross_op("s2b", s_int)(m_s)         # (3, 1, ny, M)
            cb = pre(Gb, axis=-1)
            Hb = samp(cb[:, 0], u_b)
            return Hb[:, None], Hs[:, None], F
        # scalar-potential mode
        phi = self.cross_op("b2s", s_int)(m_b)[0]          # (7, ny+6, M)
        cphi = prefilter(phi, axis=-1)

        def ptil(layer, r0, u):
            return interp_1d(cphi[layer, r0:r0 + ny], u)

        def Htil(layer, r0, u):
            # r0: window row index of slider row 0 for this evaluation
            hx = -_d4(ptil(layer, r0, u - 2), ptil(layer, r0, u - 1),
                      ptil(layer, r0, u + 1), ptil(layer, r0, u + 2), d.dx)
            hy = -_d4(ptil(layer, r0 - 2, u), ptil(layer, r0 - 1, u),
                      ptil(layer, r0 + 1, u), ptil(layer, r0 + 2, u), d.dy)
            hz = -_d4(ptil(layer - 2, r0, u), ptil(layer - 1, r0, u),
                      ptil(layer + 1, r0, u), ptil(layer + 2, r0, u), d.dz)
            return np.array([hx, hy, hz])

        Hs = Htil(3, 3, u_s)
        if want_force:
            ms = m_s[:, 0]
            dHdx = (Htil(3, 3, u_s + 1) - Htil(3, 3, u_s - 1)) / (2 * d.dx)
            dHdy = (Htil(3, 4, u_s) - Htil(3, 2, u_s)) / (2 * d.dy)
            dHdz = (Htil(4, 3, u_s) - Htil(2, 3, u_s)) / (2 * d.dz)
            F = MU0 * d.Ms * V * (ms[0][None] * dHdx + ms[1][None] * dHdy
                                  + ms[2][None] * dHdz).sum(axis=(1, 2))
        phib = self.cross_op("s2b", s_int)(m_s)[0]         # (5, ny+4, M)
        cb = prefilter(phib, axis=-1)

        def pb(layer, r0, u):
            return interp_1d(cb[layer, r0:r0 + ny], u)

        hx = -_d4(pb(2, 2, u_b - 2), pb(2, 2, u_b - 1), pb(2, 2, u_b + 1),
                  pb(2, 2, u_b + 2), d.dx)
        hy = -_d4(pb(2, 0, u_b), pb(2, 1, u_b), pb(2, 3, u_b), pb(2, 4, u_b),
                  d.dy)
        hz = -_d4(pb(0, 2, u_b), pb(1, 2, u_b), pb(3, 2, u_b), pb(4, 2, u_b),
                  d.dz)
        Hb = np.array([hx, hy, hz])
        return Hb[:, None], Hs[:, None], F

    def base_field_stencil(self, m_b, x, s_int):
        """The base film's field sampled on the slider's shifted lattice:
        at the slider cells ("c") and at their six neighbour points
        (x+-1: "xp"/"xm", y+-1: "yp"/"ym", layers z_s+-1: "zp"/"zm"), each
        (3, ny, nx) [A/m].  The points of Eq. 3's differences and of Eq. 13's
        divergence and curl."""
        d = self.desc
        h, ny = d.halo, d.ny
        xp = x / d.dx - s_int
        u_s = np.arange(d.nx, dtype=np.float64) + h + xp
        if d.cross_mode in (0, 2):
            pre = prefilter if d.cross_mode == 0 else (lambda G, axis: G)
            samp = interp_1d if d.cross_mode == 0 else linear_1d
            c = pre(self.cross_op("b2s", s_int)(m_b), axis=-1)   # (3, 3, ny+2, M)
            return {"c": samp(c[:, 1, 1:ny + 1], u_s),
                    "xp": samp(c[:, 1, 1:ny + 1], u_s + 1), "xm": samp(c[:, 1, 1:ny + 1], u_s - 1),
                    "yp": samp(c[:, 1, 2:ny + 2], u_s), "ym": samp(c[:, 1, 0:ny], u_s),
                    "zp": samp(c[:, 2, 1:ny + 1], u_s), "zm": samp(c[:, 0, 1:ny + 1], u_s)}
        cphi = prefilter(self.cross_op("b2s", s_int)(m_b)[0], axis=-1)

        def ptil(layer, r0, u):
            return interp_1d(cphi[layer, r0:r0 + ny], u)

        def Htil(layer, r0, u):
            hx = -_d4(ptil(layer, r0, u - 2), ptil(layer, r0, u - 1),
                      ptil(layer, r0, u + 1), ptil(layer, r0, u + 2), d.dx)
            hy = -_d4(ptil(layer, r0 - 2, u), ptil(layer, r0 - 1, u),
                      ptil(layer, r0 + 1, u), ptil(layer, r0 + 2, u), d.dy)
            hz = -_d4(ptil(layer - 2, r0, u), ptil(layer - 1, r0, u),
                      ptil(layer + 1, r0, u), ptil(layer + 2, r0, u), d.dz)
            return np.array([hx, hy, hz])

        return {"c": Htil(3, 3, u_s), "xp": Htil(3, 3, u_s + 1), "xm": Htil(3, 3, u_s - 1),
                "yp": Htil(3, 4, u_s), "ym": Htil(3, 2, u_s),
                "zp": Htil(4, 3, u_s), "zm": Htil(2, 3, u_s)}

    # ------------------------------------------------------------- fields
    def field_terms(self, m_list=None, x=None, s_int=None, want_force=True):
        """Per-film dict of H_eff terms [A/m] and the slider force [N]."""
        d = self.desc
        m_list = self.m if m_list is None else m_list
        x = self.x if x is None else x
        s_int = self.s_int if s_int is None else s_int
        op = self.self_op()
        out = []
        for m in m_list:
            if d.pbc:
                from .periodic import exchange_periodic
                ex = exchange_periodic(d, m)
            else:
                ex = _fields.exchange(d, m)
            out.append({
                "exchange": ex,
                "anisotropy": _fields.anisotropy(d, m),
                "zeeman": _fields.zeeman(d, m),
                "demag_self": op(m),
                "demag_cross": np.zeros_like(m),
                "eddy": np.zeros_like(m),
            })
        if self.hext_fields[0] is not None:
            out[0]["zeeman"] = out[0]["zeeman"] + np.asarray(self.hext_fields[0], dtype=np.float64)[:, None]
        if d.n_films == 2 and self.hext_fields[1] is not None:
            from .applied import slider_samples
            out[1]["zeeman"] = out[1]["zeeman"] + slider_samples(d, self.hext_fields[1], x, s_int)[:, None]
        F = np.zeros(3)
        if d.n_films == 2:
            Hb, Hs, F = self.cross_fields(m_list[0], m_list[1], x, s_int,
                                          want_force)
            out[0]["demag_cross"] = Hb
            out[1]["demag_cross"] = Hs
            if self.base_cross is not None:
                out[0]["demag_cross"] = self.base_cross(m_list[1], x)
        if self.eddy is not None:
            out[0]["eddy"] = self.eddy.H_eddy.copy()
        return out, F

    @staticmethod
    def total(terms):
        return sum(terms[k] for k in TERMS)

    # --------------------------------------------------------- dynamics
    def rigid_rhs(self, x, v, t, F):
        dr = self.drive
        if dr.mode == FROZEN:
            return 0.0, 0.0
        if dr.mode == VELOCITY:
            return dr.v_d, 0.0
        a = (dr.k * (dr.v_d * t + dr.x_anchor0 - x) - dr.gamma_v * dr.mass * v
             + F[0]) / dr.mass
        return v, a

    def derivative(self, m_list, x, v, t):
        terms, F = self.field_terms(m_list, x, self.s_int,
                                    want_force=(self.drive.mode == SPRING))
        dm = [llg_rhs(m, self.total(tf), self.desc.alpha)
              for m, tf in zip(m_list, terms)]
        dx, dv = self.rigid_rhs(x, v, t, F)
        return dm, dx, dv

    def step(self, dt):
        """One classic RK4 step of (m, x_s, v_s), renormalise, re-seat."""
        if self.eddy is not None:
            self.eddy.update(self, dt)
        m0, x0, v0, t0 = self.m, self.x, self.v, self.t
        k1 = self.derivative(m0, x0, v0, t0)
        m2 = [m + 0.5 * dt * k for m, k in zip(m0, k1[0])]
        k2 = self.derivative(m2, x0 + 0.5 * dt * k1[1], v0 + 0.5 * dt * k1[2],
                             t0 + 0.5 * dt)
        m3 = [m + 0.5 * dt * k for m, k in zip(m0, k2[0])]
        k3 = self.derivative(m3, x0 + 0.5 * dt * k2[1], v0 + 0.5 * dt * k2[2],
                             t0 + 0.5 * dt)
        m4 = [m + dt * k for m, k in zip(m0, k3[0])]
        k4 = self.derivative(m4, x0 + dt * k3[1], v0 + dt * k3[2], t0 + dt)
        new = []
        for f in range(len(m0)):
            mn = m0[f] + dt / 6.0 * (k1[0][f] + 2 * k2[0][f] + 2 * k3[0][f]
                                     + k4[0][f])
            new.append(mn / np.sqrt((mn * mn).sum(axis=0, keepdims=True)))
        self.m = new
        self.x = x0 + dt / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        self.v = v0 + dt / 6.0 * (k1[2] + 2 * k2[2] + 2 * k3[2] + k4[2])
        self.t = t0 + dt
        self.s_int = int(math.floor(self.x / self.desc.dx))
        self.step_count += 1

    def run(self, dt, n):
        for _ in range(n):
            self.step(dt)

    # ------------------------------------------------------ diagnostics
    def force(self):
        """Eq. (3) force on the slider [N] at the current state."""
        _, F = self.field_terms(want_force=True)
        return F

    def energies(self, m_list=None, x=None):
        """Energy terms [J] with the interpolated cross field (Sec. III)."""
        d = self.desc
        m_list = self.m if m_list is None else m_list
        terms, _ = self.field_terms(m_list, x, want_force=False)
        V = d.dx * d.dy * d.dz
        e = dict(exchange=0.0, anisotropy=0.0, zeeman=0.0, demag_self=0.0,
                 demag_cross=0.0)
        u = np.asarray(d.u, dtype=np.float64)
        for f, (m, tf) in enumerate(zip(m_list, terms)):
            e["exchange"] += -0.5 * MU0 * d.Ms * V * np.sum(m * tf["exchange"])
            mu = np.einsum("a...,a->...", m, u)
            e["anisotropy"] += d.Ku * V * np.sum(1.0 - mu * mu)
            e["zeeman"] += -MU0 * d.Ms * V * np.sum(m * tf["zeeman"])
            e["demag_self"] += -0.5 * MU0 * d.Ms * V * np.sum(m * tf["demag_self"])
        if d.n_films == 2:
            e["demag_cross"] = -MU0 * d.Ms * V * np.sum(
                m_list[1] * terms[1]["demag_cross"])
        e["total"] = sum(e.values())
        return e

    def p_diss(self, m_list=None):
        """Eq. (4): gamma alpha mu0 V Ms / (1+alpha^2) sum |m x H_eff|^2."""
        d = self.desc
        m_list = self.m if m_list is None else m_list
        terms, _ = self.field_terms(m_list, want_force=False)
        V = d.dx * d.dy * d.dz
        s = 0.0
        for m, tf in zip(m_list, terms):
            mxh = np.cross(m, self.total(tf), axis=0)
            s += np.sum(mxh * mxh)
        return GAMMA0 * d.alpha * MU0 * V * d.Ms / (1 + d.alpha ** 2) * s
