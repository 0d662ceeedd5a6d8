"""GPU step paths beyond the field tests: the slider crossing cell
boundaries (the re-seat of Sec. III: s_int = floor(x_s / dx) after the step,
which moves the spline windows and the force rows), the constant-velocity
and spring drives of Eq. 15, the watchdog flags raised while stepping, and
drive changes on batch instances.  Every trajectory is compared with the
float64 oracle every 20 steps: max |dm| over all cells of both films, the
slider position and velocity."""
import math
import numpy as np
import pytest

from workloads import Desc, Drive, slider_mass_damping
from workloads.states import domain_state
from gpu_common import oracle_system

pytestmark = pytest.mark.gpu

TOL_M = {32: 1e-4, 64: 1e-9}


def films(prec, nx=48, ny=20, travel=3):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=1,
             max_travel_cells=travel, Ms=1.1e6, Aex=1.5e-11, alpha=0.1, Ku=8e5, precision=prec)
    m = [domain_state((1, ny, nx), 31), domain_state((1, ny, nx), 32)]
    return d, m


def track(desc, drive, m, dt, nsteps, every=20):
    import torch
    import paper_1801_04181_amd as mmv
    mesh = mmv.Mesh(desc, drive, m)
    s = oracle_system(desc, drive, m)
    seats = {s.s_int}
    worst = 0.0
    for k in range(nsteps // every):
        mesh.step(dt, every)
        torch.cuda.synchronize()
        s.run(dt, every)
        seats.add(s.s_int)
        st = mesh.state()
        dm = max(np.abs(mesh.get_m(f).cpu().numpy() - s.m[f]).max() for f in range(2))
        ex = abs(st["x"] - s.x) / desc.dx
        ev = abs(st["v"] - s.v)
        print(f"  step {(k + 1) * every}: x {st['x'] / desc.dx:.6f} cells (oracle {s.x / desc.dx:.6f}, "
              f"s_int {s.s_int}) max|dm| {dm:.2e} dx {ex:.2e} dv {ev:.2e}", flush=True)
        worst = max(worst, dm)
        assert dm <= TOL_M[desc.precision], (k, dm)
        assert ex <= 1e-4, (k, ex)
        assert ev <= 1e-4 * max(abs(s.v), 1e-3), (k, ev)
        assert math.floor(st["x"] / desc.dx) == s.s_int
    mesh.close()
    return seats, worst


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("v,x0", [(5.0, 0.98), (-5.0, 0.02)])
def test_velocity_drive_crosses_a_cell_boundary(prec, v, x0):
    """The slider moves 2.5e-4 cell per step: it crosses x = 1 (v > 0) or
    x = 0 (v < 0) at step 80 of 200."""
    d, m = films(prec)
    print(f"velocity drive {v} m/s from {x0} cell, fp{prec}", flush=True)
    seats, worst = track(d, Drive(mode=1, v_d=v, x0=x0 * d.dx), m, 1e-13, 200)
    assert seats == ({0, 1} if v > 0 else {0, -1})


@pytest.mark.parametrize("prec", [32, 64])
def test_spring_drive_crosses_a_cell_boundary(prec):
    """Spring drive (Eq. 15) started at 0.98 cell moving at the anchor's 5
    m/s with the spring relaxed: the force of Eq. 3 and the spring act
    while the slider re-seats."""
    d, m = films(prec)
    mass, gv = slider_mass_damping(d.nx, d.ny, 1e-3)
    x0 = 0.98 * d.dx
    drv = Drive(mode=2, v_d=5.0, k=1e-3, mass=mass, gamma_v=gv, x_anchor0=x0, x0=x0, v0=5.0)
    print(f"spring drive from 0.98 cell, fp{prec}", flush=True)
    seats, worst = track(d, drv, m, 1e-13, 200)
    assert 1 in seats


def test_stepping_out_of_the_window_reports_erange():
    import torch
    import paper_1801_04181_amd as mmv
    d, m = films(32, nx=24, ny=8, travel=1)
    mesh = mmv.Mesh(d, Drive(mode=1, v_d=5.0, x0=1.99 * d.dx), m)
    assert mesh.state()["step"] == 0
    print("velocity drive past max_travel_cells = 1", flush=True)
    mesh.step(1e-13, 60)          # x reaches 2 cells at step 40
    torch.cuda.synchronize()
    with pytest.raises(mmv.MMVError) as e:
        mesh.state()
    assert e.value.code == -4
    mesh.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_non_finite_magnetisation_reports_enumeric(prec):
    import torch
    import paper_1801_04181_amd as mmv
    d, m = films(prec, nx=24, ny=8)
    bad = [x.copy() for x in m]
    bad[0][1, 0, 3, 5] = float("nan")
    mesh = mmv.Mesh(d, Drive(), m)
    mesh.step(1e-13, 2)
    assert mesh.state()["step"] == 2
    mesh.set_m(0, bad[0])
    print(f"NaN in film 0, fp{prec}", flush=True)
    mesh.step(1e-13, 1)
    torch.cuda.synchronize()
    with pytest.raises(mmv.MMVError) as e:
        mesh.state()
    assert e.value.code == -5
    mesh.close()


def test_set_drive_on_a_batch_instance_takes_effect():
    """A batch instance whose spring speed changes between batch_step calls
    follows the same trajectory, bit for bit, as a single mesh given the
    same sequence."""
    import torch
    import paper_1801_04181_amd as mmv
    from workloads.configs import batch_pairs
    pairs = batch_pairs(4)
    for p in pairs:
        p["desc"] = p["desc"].replace(nx=p["desc"].nx // 4, ny=p["desc"].ny // 4)
    from workloads import initial_state
    ms = [initial_state(p) for p in pairs]
    B = mmv.Batch([p["desc"] for p in pairs], [p["drive"] for p in pairs], ms)
    i = 2
    single = mmv.Mesh(pairs[i]["desc"], pairs[i]["drive"], ms[i])
    cur = pairs[i]["drive"]
    for v_new in (3.0, 0.5):
        B.step(1e-13, 12)
        single.step(1e-13, 12)
        torch.cuda.synchronize()
        st = single.state()
        assert B.state(i) == st
        # new anchor speed, anchor position continuous at the current time
        anchor = cur.v_d * st["t"] + cur.x_anchor0
        cur = Drive(**{**cur.__dict__, "v_d": v_new, "x_anchor0": anchor - v_new * st["t"],
                       "x0": st["x"], "v0": st["v"]})
        for h in (B.h[i], single.h):
            mmv.set_drive(h, cur)
    B.step(1e-13, 12)
    single.step(1e-13, 12)
    torch.cuda.synchronize()
    sb, s1 = B.state(i), single.state()
    print("batch instance", sb, "single", s1, flush=True)
    assert sb == s1
    for f in range(2):
        assert torch.equal(B.get_m(i, f), single.get_m(f)), f
    # the new drive really acts: the spring anchor now moves at 0.5 m/s
    ref = mmv.Mesh(pairs[i]["desc"], pairs[i]["drive"], ms[i])
    ref.step(1e-13, 36)
    torch.cuda.synchronize()
    assert ref.state()["x"] != sb["x"]
    ref.close()
    single.close()
    B.close()
