"""Write the oracle's 2000-step run of the 64^3 conducting cube, sampled.

Runs only the float64 oracle (oracle/) on the seeded synthetic cube of
workloads/ (eddy currents on, RK4 dt 5e-14 s) and stores, every 500 steps,
the magnetisation on the strided sub-lattice of every fourth cell along each
axis (16^3 cells) and the mean magnetisation of the whole cube:

  cube_2000.npz   m_<step> (3, 16, 16, 16) float64, mean_<step> (3,),
                  steps = (500, 1000, 1500, 2000)

About three hours on one core.  Used by tests/precision_report.py (the
long-run float32/float64 drift against the oracle).  Usage:
  python tests/golden/make_cube_long.py
"""
import os
import sys
import time
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import get_config, initial_state  # noqa: E402
from oracle.sim import System  # noqa: E402

STEPS = (500, 1000, 1500, 2000)
STRIDE = 4


def main():
    cfg = get_config("cube_eddy")
    d = cfg["desc"].replace(precision=64)
    s = System(d, cfg["drive"], initial_state(cfg))
    out = {"steps": np.array(STEPS), "stride": STRIDE}
    t0 = time.time()
    for n in range(STEPS[-1]):
        s.step(cfg["dt"])
        if (n + 1) % 50 == 0:
            print("cube step", n + 1, f"{time.time() - t0:.0f} s", flush=True)
        if n + 1 in STEPS:
            m = s.m[0]
            out[f"m_{n + 1}"] = m[:, ::STRIDE, ::STRIDE, ::STRIDE].copy()
            out[f"mean_{n + 1}"] = m.reshape(3, -1).mean(axis=1)
            np.savez_compressed(os.path.join(HERE, "cube_2000.npz"), **out)


if __name__ == "__main__":
    main()
