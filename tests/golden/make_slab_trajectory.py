"""Write the oracle's 1000-step run of two thick conducting films.

Runs only the float64 oracle (oracle/slab.py) on the seeded synthetic case
below (two films of 16 x 12 x 3 cells of 4 nm, one cell apart, CoCrPt with
sigma = 1e6 S/m, stripes five cells wide, 20 SOR sweeps per step, the slider
driven at 60 m/s from 0.3 cell so that it crosses a cell boundary near step
470; RK4 dt 1e-13 s) and stores, every 250 steps, both films' magnetisation,
the slider's position and velocity, and at the end each film's eddy field:

  slab_1000.npz   m0_<step>, m1_<step> (3, 3, 12, 16) float64,
                  x_<step>, v_<step>, eddy0, eddy1 (3, 3, 12, 16),
                  steps = (250, 500, 750, 1000)

About a minute on one core.  With --periodic, the same films periodic in
x and y (one image on each side), the slider driven from 15.3 cells so that
it crosses the period (s_int 15 -> 16 = nx) near step 470:

  slab_periodic_1000.npz   the same keys

Used by tests/test_gpu_slab.py.  Usage:
  python tests/golden/make_slab_trajectory.py [--periodic]
"""
import os
import sys
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import Desc, Drive  # noqa: E402
from workloads.states import stripe_state  # noqa: E402
from oracle.slab import SlabSystem  # noqa: E402

STEPS = (250, 500, 750, 1000)
DT = 1e-13


def case(precision=64, periodic=False):
    """Descriptor, drive and initial state of the stored run."""
    d = Desc(n_films=2, nx=16, ny=12, nz=3, dx=4e-9, dy=4e-9, dz=4e-9, gap_cells=1, max_travel_cells=4,
             Ms=3.5e5, Aex=5e-12, alpha=0.05, Ku=1.225e5, u=(0.0, 0.0, 1.0), sigma=1e6, precision=precision,
             halo=4, sor_sweeps=20)
    m = [stripe_state((3, 12, 16), 31 + f, width_cells=5) for f in range(2)]
    if periodic:
        d = d.replace(pbc=3, pbc_images=1)
        return d, Drive(mode=1, v_d=60.0, x0=15.3 * d.dx), m
    return d, Drive(mode=1, v_d=60.0, x0=0.3 * d.dx), m


def main(periodic=False):
    d, drv, m = case(periodic=periodic)
    s = SlabSystem(d, drv, m)
    out = {"steps": np.array(STEPS)}
    for n in range(STEPS[-1]):
        s.step(DT)
        if n + 1 in STEPS:
            out[f"m0_{n + 1}"] = s.m[0].copy()
            out[f"m1_{n + 1}"] = s.m[1].copy()
            out[f"x_{n + 1}"] = s.x
            out[f"v_{n + 1}"] = s.v
            print("slab step", n + 1, "x/dx", s.x / d.dx, flush=True)
    out["eddy0"] = s.eddy.H[0].copy()
    out["eddy1"] = s.eddy.H[1].copy()
    name = "slab_periodic_1000.npz" if periodic else "slab_1000.npz"
    np.savez_compressed(os.path.join(HERE, name), **out)


if __name__ == "__main__":
    main(periodic="--periodic" in sys.argv[1:])
