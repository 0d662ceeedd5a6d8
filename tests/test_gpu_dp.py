"""Adaptive Dormand-Prince runs (the paper's RK45 solver with the slider's
equation of motion, Sec. III) on the GPU against the float64 oracle's run
(oracle/dormand_prince.py) from the same state, tolerance and first step.

float64: the accept/reject decisions are threshold tests of the error ratio,
which both sides compute to ~1e-12, so the runs take the same steps: equal
accepted and rejected counts, m within 1e-9, slider within 1e-9 cell.
float32: the ratio carries float32 rounding, so a decision near the threshold
may go the other way; both runs stay within the tolerance of the exact
trajectory, so the final states agree to a few times the tolerance
(bar 1e-4 on m, the trajectory bar) and the counts to within a few steps.
"""
import math
import numpy as np
import pytest

from workloads import Desc, Drive, get_config, initial_state, slider_mass_damping
from workloads.states import domain_state
from gpu_common import oracle_system

pytestmark = pytest.mark.gpu


def run_both(desc, drive, m, t_end, tol, h0):
    import torch
    import paper_1801_04181_amd as mmv
    from oracle import dormand_prince as dp
    print(f"dp run {desc.nx}x{desc.ny} fp{desc.precision} to {t_end:g} s, tol {tol:g}", flush=True)
    mesh = mmv.Mesh(desc, drive, m)
    g = mesh.run_dp(t_end, tol, h0)
    torch.cuda.synchronize()
    s = oracle_system(desc, drive, m)
    acc, rej, h_or = dp.run(s, t_end, h0, tol)
    st = mesh.state()
    dm = max(np.abs(mesh.get_m(f).cpu().numpy() - s.m[f]).max() for f in range(desc.n_films))
    out = dict(gpu=g, oracle=dict(accepted=acc, rejected=rej, h=h_or), dm=dm,
               dx=abs(st["x"] - s.x) / desc.dx, t=(st["t"], s.t), step=st["step"])
    print("  ", out, flush=True)
    mesh.close()
    return out


def test_tiny_fp64_same_steps_as_the_oracle():
    cfg = get_config("tiny")
    r = run_both(cfg["desc"], cfg["drive"], initial_state(cfg), 2e-12, 1e-6, 1e-12)
    assert r["gpu"]["accepted"] == r["oracle"]["accepted"]
    assert r["gpu"]["rejected"] == r["oracle"]["rejected"]
    assert r["gpu"]["accepted"] > 5 and r["gpu"]["rejected"] >= 1   # the 1e-12 s first step fails
    assert r["t"][0] == r["t"][1] == 2e-12
    assert r["step"] == r["gpu"]["accepted"]
    assert r["dm"] < 1e-9
    assert r["gpu"]["h"] == pytest.approx(r["oracle"]["h"], rel=1e-9)


def spring_films(prec, nx=48, ny=20):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=1,
             max_travel_cells=3, Ms=1.1e6, Aex=1.5e-11, alpha=0.1, Ku=8e5, precision=prec)
    m = [domain_state((1, ny, nx), 51), domain_state((1, ny, nx), 52)]
    mass, gv = slider_mass_damping(nx, ny, 1e-3)
    x0 = 0.98 * d.dx
    drv = Drive(mode=2, v_d=20.0, k=1e-3, mass=mass, gamma_v=gv, x_anchor0=x0, x0=x0, v0=20.0)
    return d, drv, m


def test_spring_fp64_crossing_a_cell_boundary():
    """Spring drive at 20 m/s from 0.98 cell: the slider re-seats during the
    run (x passes 1 cell after about 1e-12 s)."""
    d, drv, m = spring_films(64)
    r = run_both(d, drv, m, 3e-12, 1e-6, 1e-14)
    assert r["gpu"]["accepted"] == r["oracle"]["accepted"]
    assert r["gpu"]["rejected"] == r["oracle"]["rejected"]
    assert r["dm"] < 1e-9
    assert r["dx"] < 1e-9


def test_spring_fp32_within_the_tolerance():
    d, drv, m = spring_films(32, nx=96, ny=40)
    r = run_both(d, drv, m, 3e-12, 1e-5, 1e-14)
    assert r["dm"] < 1e-4
    assert r["dx"] < 1e-4
    assert abs(r["gpu"]["accepted"] - r["oracle"]["accepted"]) <= 3


def test_run_validation_and_attempt_limit():
    import torch
    import paper_1801_04181_amd as mmv
    cfg = get_config("tiny")
    mesh = mmv.Mesh(cfg["desc"], cfg["drive"], initial_state(cfg))
    with pytest.raises(mmv.MMVError) as e:
        mesh.run_dp(0.0, 1e-6, 1e-14)          # t_end not after t = 0
    assert e.value.code == -1
    with pytest.raises(mmv.MMVError) as e:
        mesh.run_dp(1e-12, 0.0, 1e-14)
    assert e.value.code == -1
    r = mesh.run_dp(1e-11, 1e-6, 1e-14, max_attempts=3)
    assert r["accepted"] + r["rejected"] == 3
    st = mesh.state()
    assert 0.0 < st["t"] < 1e-11 and st["step"] == r["accepted"]
    # the run continues from there, and plain RK4 steps afterwards still work
    r2 = mesh.run_dp(2e-13 + st["t"], 1e-6, r["h"])
    assert mesh.state()["t"] == pytest.approx(2e-13 + st["t"], rel=1e-12)
    mesh.step(1e-14, 2)
    torch.cuda.synchronize()
    assert mesh.state()["step"] == r["accepted"] + r2["accepted"] + 2
    mesh.close()
    cube = get_config("cube_eddy")["desc"].replace(nx=8, ny=8, nz=8)
    c = mmv.Mesh(cube, Drive())
    with pytest.raises(mmv.MMVError) as e:
        c.run_dp(1e-12, 1e-6, 1e-14)
    assert e.value.code == -6
    c.close()
