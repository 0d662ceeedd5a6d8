"""Problem description shared by both sides (plain data, SI units)."""
from dataclasses import dataclass, field, replace
import math

MU0 = 4e-7 * math.pi

# Drive modes of the slider (Sec. III, Eq. 15).
DRIVE_FROZEN = 0      # slider held at its initial position
DRIVE_VELOCITY = 1    # slider moved at constant velocity v_d
DRIVE_SPRING = 2      # slider pulled by a spring whose anchor moves at v_d


@dataclass
class Drive:
    mode: int = DRIVE_FROZEN
    v_d: float = 0.0          # anchor (or slider) velocity [m/s]
    k: float = 0.0            # spring constant [N/m]
    mass: float = 1.0         # slider mass [kg]
    gamma_v: float = 0.0      # viscous damping coefficient [1/s] (Eq. 14)
    x_anchor0: float = 0.0    # anchor position at t=0 [m]
    x0: float = 0.0           # slider position at t=0 [m]
    v0: float = 0.0           # slider velocity at t=0 [m/s]


@dataclass
class Desc:
    n_films: int = 2          # 1: single magnet; 2: base (film 0) + slider (film 1)
    nx: int = 32
    ny: int = 32
    nz: int = 1
    dx: float = 5e-9
    dy: float = 5e-9
    dz: float = 5e-9
    gap_cells: int = 1        # empty layers between base and slider
    max_travel_cells: int = 2 # |s_int| bound that sizes the FFT window
    Ms: float = 8e5
    Aex: float = 1.3e-11
    alpha: float = 0.5
    Ku: float = 0.0
    u: tuple = (0.0, 0.0, 1.0)
    Hext: tuple = (0.0, 0.0, 0.0)
    sigma: float = 0.0        # conductivity [S/m]; 0 disables eddy currents
    precision: int = 32       # 32 or 64
    cross_mode: int = 0       # 0 direct field spline, 1 scalar potential, 2 direct field, linear interpolation
    halo: int = 4             # spline window extension along the motion axis
    rc_cells: float = 30.0    # Newell / point-dipole switch radius [cells]
    sor_sweeps: int = 0       # fixed red-black SOR sweeps per step (0: library default)
    sor_omega: float = 0.0    # SOR relaxation factor (0: 2/(1+sin(pi/n_max)))
    pbc: int = 0              # periodic in-plane axes: bit 0 = x, bit 1 = y (one- and two-layer films)
    pbc_images: int = 0       # periodic images summed on each side per periodic axis

    @property
    def z_s(self):
        """z-layer index of the slider relative to the base."""
        return self.nz + self.gap_cells

    @property
    def cells(self):
        return self.n_films * self.nx * self.ny * self.nz

    def replace(self, **kw):
        return replace(self, **kw)
