"""Write the oracle's 1000-step trajectories of two workloads.

Runs only the float64 oracle (oracle/) on the seeded synthetic inputs of
workloads/ and stores, after 1000 RK4 steps, the full magnetisation of both
films (float64) and the slider state:

  stickslip_1000.npz  2 films 512 x 128, spring drive, dt 1e-13 s
                      (about 10 minutes on one core)
  tiny_1000.npz       2 films 32 x 32, 5 nm, slider frozen at 0.37 cell,
                      dt 1e-13 s (about a minute)

Used by tests/test_gpu_trajectory.py.  Usage:
  python tests/golden/make_trajectories.py [stickslip|tiny ...]
"""
import os
import sys
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import get_config, initial_state  # noqa: E402
from oracle.sim import System  # noqa: E402

STEPS = 1000


def make(name):
    cfg = get_config(name)
    s = System(cfg["desc"], cfg["drive"], initial_state(cfg))
    for n in range(STEPS):
        s.step(cfg["dt"])
        if (n + 1) % 100 == 0:
            print(name, "step", n + 1, "x", s.x, flush=True)
    out = os.path.join(HERE, f"{name}_1000.npz")
    np.savez_compressed(out, m0=s.m[0], m1=s.m[1], x=s.x, v=s.v, t=s.t,
                        s_int=s.s_int, steps=STEPS)


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["tiny", "stickslip"]):
        make(name)
