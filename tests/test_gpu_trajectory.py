"""1000 RK4 steps on the GPU against the stored float64 oracle trajectories
(tests/golden/*_1000.npz, written by make_trajectories.py from the oracle
alone):

  stickslip  2 x 512 x 128 films, spring drive, float32 and float64
  tiny       2 x 32 x 32 films, slider frozen at 0.37 cell, float64

Bars: max over every cell of both films of |m_gpu - m_oracle| <= 1e-4 in
float32 (the trajectory bar) and 1e-8 in float64; slider position within
1e-5 cell (float32) / 1e-9 cell (float64).  The per-step float32 error of H
is ~1e-7 relative and the damped dynamics do not amplify it beyond linear
growth.
"""
import os
import numpy as np
import pytest

from workloads import get_config, initial_state

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name,precision,tol,tol_x", [
    ("stickslip", 32, 1e-4, 1e-5), ("stickslip", 64, 1e-8, 1e-9), ("tiny", 64, 1e-8, 1e-9)])
def test_thousand_steps_match_oracle_trajectory(name, precision, tol, tol_x):
    import torch
    import paper_1801_04181_amd as mmv
    g = np.load(os.path.join(GOLDEN, f"{name}_1000.npz"))
    cfg = get_config(name)
    d = cfg["desc"].replace(precision=precision)
    print(f"trajectory {name} fp{precision}", flush=True)
    me = mmv.Mesh(d, cfg["drive"], initial_state(cfg))
    steps = int(g["steps"])
    for _ in range(steps // 100):
        me.step(cfg["dt"], 100)
    torch.cuda.synchronize()
    for f, key in enumerate(("m0", "m1")):
        got = me.get_m(f).cpu().numpy()
        ref = g[key]
        assert got.shape == ref.shape
        drift = np.abs(got - ref).max()
        print(f"film {f} max |dm| {drift:.3e}", flush=True)
        assert drift <= tol
    st = me.state()
    assert st["step"] == steps
    assert abs(st["t"] - float(g["t"])) <= 1e-12 * float(g["t"])
    dxc = abs(st["x"] - float(g["x"])) / d.dx
    print(f"slider x error {dxc:.3e} cells", flush=True)
    assert dxc <= tol_x
    me.close()
