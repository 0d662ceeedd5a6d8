"""The five synthetic workloads (plus the gap-3 potential-mode variant).

Material constants and drives are the ones named for each workload; where
the paper leaves a parameter open (slider mass, viscous damping, time step)
the choice is written here once and used by both sides.
"""
import math
from .desc import Desc, Drive, DRIVE_FROZEN, DRIVE_SPRING, DRIVE_VELOCITY, MU0


def slider_mass_damping(nx, ny, k):
    """Slider mass scaled with its area and critical viscous damping.

    The paper only asks for a critically damped spring-slider whose viscous
    force at v_d is well below the magnetic force (Sec. IV.B, Eqs. 14-15).
    Mass 1e-20 kg per 256x256 cells; gamma_v = 2 sqrt(k/m).
    """
    mass = 1e-20 * (nx * ny / 65536.0)
    gamma_v = 2.0 * math.sqrt(k / mass) if k > 0 else 0.0
    return mass, gamma_v


def _cfg_tiny(gap=1, cross_mode=0):
    d = Desc(n_films=2, nx=32, ny=32, nz=1, dx=5e-9, dy=5e-9, dz=5e-9,
             gap_cells=gap, max_travel_cells=0, Ms=8e5, Aex=1.3e-11,
             alpha=0.5, Ku=0.0, precision=64, cross_mode=cross_mode)
    drv = Drive(mode=DRIVE_FROZEN, x0=0.37 * 5e-9)
    return dict(desc=d, drive=drv, dt=1e-13, steps=100, seed=1801,
                state="random")


def _cfg_stickslip():
    d = Desc(n_films=2, nx=512, ny=128, nz=1, dx=2e-9, dy=2e-9, dz=2e-9,
             gap_cells=1, max_travel_cells=8, Ms=1.1e6, Aex=1.5e-11,
             alpha=0.1, Ku=8e5, u=(0.0, 0.0, 1.0), precision=32)
    mass, gv = slider_mass_damping(512, 128, 1e-3)
    drv = Drive(mode=DRIVE_SPRING, v_d=1.0, k=1e-3, mass=mass, gamma_v=gv)
    return dict(desc=d, drive=drv, dt=1e-13, steps=20000, seed=(2, 3),
                state="domains")


def _cfg_cube():
    d = Desc(n_films=1, nx=64, ny=64, nz=64, dx=2e-9, dy=2e-9, dz=2e-9,
             gap_cells=0, max_travel_cells=0, Ms=8e5, Aex=1.3e-11,
             alpha=0.01, Ku=0.0, Hext=(0.0, 0.0, -0.05 / MU0), sigma=1e7,
             precision=32)
    return dict(desc=d, drive=Drive(), dt=5e-14, steps=2000, seed=33,
                state="cube")


def batch_pairs(n=64, seed=4):
    """The uneven batch: pair i has nx={64,128,256,512}[i%4], ny={64,128}[(i//4)%2]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.1, 5.0, size=n)
    out = []
    for i in range(n):
        nx = (64, 128, 256, 512)[i % 4]
        ny = (64, 128)[(i // 4) % 2]
        d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=2e-9, dz=2e-9,
                 gap_cells=1, max_travel_cells=4, Ms=1.1e6, Aex=1.5e-11,
                 alpha=0.1, Ku=8e5, precision=32)
        mass, gv = slider_mass_damping(nx, ny, 1e-3)
        drv = Drive(mode=DRIVE_SPRING, v_d=float(v[i]), k=1e-3, mass=mass,
                    gamma_v=gv)
        out.append(dict(desc=d, drive=drv, dt=1e-13, steps=1000,
                        seed=(2 + 100 * (i + 1), 3 + 100 * (i + 1)),
                        state="domains"))
    return out


def _cfg_learned():
    d = Desc(n_films=2, nx=256, ny=256, nz=1, dx=2e-9, dy=2e-9, dz=2e-9,
             gap_cells=1, max_travel_cells=4, Ms=1.1e6, Aex=1.5e-11,
             alpha=0.1, Ku=8e5, precision=32)
    mass, gv = slider_mass_damping(256, 256, 1e-3)
    drv = Drive(mode=DRIVE_SPRING, v_d=1.0, k=1e-3, mass=mass, gamma_v=gv)
    return dict(desc=d, drive=drv, dt=1e-13, steps=10000, seed=(5, 6),
                state="domains")


def _cfg_eddy_films():
    """Two CoCrPt films 512 nm x 512 nm x 20 nm in 4 nm cells, 20 nm apart,
    conductivity 1e6 S/m, stripes ~80 nm wide, spring drive at 2 m/s with
    k = 0.005 N/m (the paper's eddy-current friction test, Sec. IV.C, on the
    material and drive of Sec. IV.B); open in-plane boundaries."""
    d = Desc(n_films=2, nx=128, ny=128, nz=5, dx=4e-9, dy=4e-9, dz=4e-9,
             gap_cells=5, max_travel_cells=8, Ms=3.5e5, Aex=5e-12,
             alpha=0.05, Ku=1.225e5, u=(0.0, 0.0, 1.0), sigma=1e6,
             precision=32)
    mass, gv = slider_mass_damping(128, 128, 0.005)
    drv = Drive(mode=DRIVE_SPRING, v_d=2.0, k=0.005, mass=mass, gamma_v=gv)
    return dict(desc=d, drive=drv, dt=1e-13, steps=1000, seed=(7, 8),
                state="stripes")


CONFIGS = {
    "tiny": _cfg_tiny,                                     # 2x 32x32x1, FP64
    "tiny_potential": lambda: _cfg_tiny(gap=3, cross_mode=1),
    "stickslip": _cfg_stickslip,                           # 2x 512x128x1, FP32
    "cube_eddy": _cfg_cube,                                # 64^3 + eddy
    "learned": _cfg_learned,                               # 2x 256x256x1
    "eddy_films": _cfg_eddy_films,                         # 2x 128x128x5 + eddy
}


def get_config(name):
    return CONFIGS[name]()
