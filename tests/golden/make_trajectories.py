"""Write the oracle's 1000-step trajectory of the stick-slip workload.

Runs only the float64 oracle (oracle/) on the seeded synthetic input of
workloads/ (2 films 512 x 128, spring drive, dt 1e-13 s) and stores the
slider state and the magnetisation on a fixed subsample of cells
((i + 3 j) mod 7 == 0) after 1000 RK4 steps.  Used by
tests/test_gpu_trajectory.py.  Takes about 10 minutes on one core.
"""
import os
import sys
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import get_config, initial_state  # noqa: E402
from oracle.sim import System  # noqa: E402

STEPS = 1000


def sample_mask(ny, nx):
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return (i + 3 * j) % 7 == 0


def main(out=os.path.join(HERE, "stickslip_1000.npz")):
    cfg = get_config("stickslip")
    s = System(cfg["desc"], cfg["drive"], initial_state(cfg))
    for n in range(STEPS):
        s.step(cfg["dt"])
        if (n + 1) % 100 == 0:
            print("step", n + 1, "x", s.x, flush=True)
    mask = sample_mask(cfg["desc"].ny, cfg["desc"].nx)
    np.savez_compressed(out, m0=s.m[0][:, 0][:, mask], m1=s.m[1][:, 0][:, mask],
                        x=s.x, v=s.v, t=s.t, s_int=s.s_int, steps=STEPS)


if __name__ == "__main__":
    main()
