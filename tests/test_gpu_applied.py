"""Non-uniform applied field in the moving magnet (Sec. II.A) on the GPU
against the float64 oracle (oracle/applied.py): the Zeeman term of both
films with the field on the frame lattice, the slider sampling it at its
moved cells with the cross field's interpolant (spline, potential mode's
spline, linear; periodic x), trajectories of a moving slider through a
cell boundary, removal of the field, and batch instances."""
import math
import numpy as np
import pytest

from workloads import Desc, Drive
from workloads.states import domain_state
from gpu_common import oracle_system, TOL, max_rel

pytestmark = pytest.mark.gpu


def films(prec, mode=0, pbc=0, nx=40, ny=14, travel=3, gap=3):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=gap, max_travel_cells=travel,
             Ms=1.1e6, Aex=1.5e-11, alpha=0.1, Ku=8e5, Hext=(1e3, -2e3, 5e3), cross_mode=mode, pbc=pbc,
             pbc_images=2, precision=prec)
    m = [domain_state((1, ny, nx), 71), domain_state((1, ny, nx), 72)]
    return d, m


def frame_fields(d, seed=9):
    """A smooth random field on the frame lattice: sums of a few plane waves
    along x and y (amplitude ~1e4 A/m), for the base cells and the slider's
    layer (periodic x: whole periods of the film)."""
    from oracle.applied import slider_width
    rng = np.random.default_rng(seed)
    W = 0 if d.pbc & 1 else d.max_travel_cells + d.halo
    xs_b = np.arange(d.nx)
    xs_s = np.arange(slider_width(d)) - W
    ys = np.arange(d.ny)
    Lx = d.nx if d.pbc & 1 else 17.0

    def field(xs):
        X, Y = np.meshgrid(xs, ys)
        out = np.zeros((3, d.ny, len(xs)))
        for c in range(3):
            for _ in range(3):
                kx = 2 * np.pi * rng.integers(1, 4) / Lx
                ky = 2 * np.pi * rng.uniform(0.0, 0.3)
                out[c] += 4e3 * rng.standard_normal() * np.cos(kx * X + ky * Y + rng.uniform(0, 2 * np.pi))
        return out
    state = rng.bit_generator.state
    hb = field(xs_b)
    rng.bit_generator.state = state           # the same waves on both layers
    hs = field(xs_s)
    return hb, hs


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("mode,pbc", [(0, 0), (1, 0), (2, 0), (0, 1)])
def test_zeeman_term_with_the_applied_field(mode, pbc, prec):
    import paper_1801_04181_amd as mmv
    d, m = films(prec, mode, pbc)
    hb, hs = frame_fields(d)
    mesh = mmv.Mesh(d, Drive(), m)
    mesh.set_hext_field(0, hb)
    mesh.set_hext_field(1, hs)
    for x in (0.37, -2.6, 1.0, 2.95):
        print(f"applied field: mode {mode} pbc {pbc} fp{prec} x={x}", flush=True)
        mesh.set_offset(x)
        s = oracle_system(d, Drive(), m, x)
        s.hext_fields = [hb, hs]
        terms, _ = s.field_terms()
        for f in range(2):
            got = mesh.eval_heff(f, mmv.TERM["zeeman"]).cpu().numpy()
            ref = terms[f]["zeeman"]
            e = rel(got, ref)
            print(f"  film {f}: rel {e:.2e} max-cell {max_rel(got, ref):.2e}", flush=True)
            assert e <= TOL[prec], (f, e)
            # the other terms are untouched
            tot = mesh.eval_heff(f, mmv.TERM["all"]).cpu().numpy()
            ref_tot = System_total(terms[f])
            assert rel(tot, ref_tot) <= (1e-5 if prec == 32 else 1e-9)
    mesh.close()


def System_total(t):
    from oracle.sim import System
    return System.total(t)


@pytest.mark.parametrize("prec", [32, 64])
def test_moving_slider_in_the_applied_field(prec):
    """Velocity drive at 5 m/s from 0.98 cell: the slider crosses x = 1
    while its cells sample the frame field; m every 20 steps against the
    oracle."""
    import torch
    import paper_1801_04181_amd as mmv
    d, m = films(prec)
    hb, hs = frame_fields(d, seed=11)
    drv = Drive(mode=1, v_d=5.0, x0=0.98 * d.dx)
    mesh = mmv.Mesh(d, drv, m)
    mesh.set_hext_field(0, hb)
    mesh.set_hext_field(1, hs)
    s = oracle_system(d, drv, m)
    s.hext_fields = [hb, hs]
    dt = 1e-13
    seats = {s.s_int}
    tol = 1e-4 if prec == 32 else 1e-9
    for k in range(8):
        mesh.step(dt, 20)
        torch.cuda.synchronize()
        s.run(dt, 20)
        seats.add(s.s_int)
        dm = max(np.abs(mesh.get_m(f).cpu().numpy() - s.m[f]).max() for f in range(2))
        print(f"  step {(k + 1) * 20}: x {s.x / d.dx:.4f} cells max|dm| {dm:.2e}", flush=True)
        assert dm <= tol, (k, dm)
    assert seats == {0, 1}
    mesh.close()


def test_removing_the_field_restores_the_uniform_result():
    import paper_1801_04181_amd as mmv
    d, m = films(32)
    hb, hs = frame_fields(d)
    mesh = mmv.Mesh(d, Drive(), m)
    mesh.set_offset(0.4)
    before = [mesh.eval_heff(f, mmv.TERM["zeeman"]).cpu().numpy() for f in range(2)]
    mesh.set_hext_field(0, hb)
    mesh.set_hext_field(1, hs)
    with_f = [mesh.eval_heff(f, mmv.TERM["zeeman"]).cpu().numpy() for f in range(2)]
    assert all(not np.array_equal(a, b) for a, b in zip(before, with_f))
    mesh.set_hext_field(0, None)
    mesh.set_hext_field(1, None)
    after = [mesh.eval_heff(f, mmv.TERM["zeeman"]).cpu().numpy() for f in range(2)]
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
    mesh.close()


def test_batch_instance_with_the_applied_field_equals_the_single_mesh():
    import torch
    import paper_1801_04181_amd as mmv
    d, m = films(32)
    hb, hs = frame_fields(d)
    drv = Drive(mode=1, v_d=3.0, x0=0.5 * d.dx)
    B = mmv.Batch([d, d], [drv, drv], [m, m])
    B.step(1e-13, 2)                         # descriptors built without the field
    single = mmv.Mesh(d, drv, m)
    single.step(1e-13, 2)
    h1 = B.h[1]
    t_b = torch.as_tensor(hb, dtype=torch.float32).cuda().contiguous()
    t_s = torch.as_tensor(hs, dtype=torch.float32).cuda().contiguous()
    mmv.set_hext_field(h1, 0, t_b)
    mmv.set_hext_field(h1, 1, t_s)
    single.set_hext_field(0, hb)
    single.set_hext_field(1, hs)
    torch.cuda.synchronize()
    B.step(1e-13, 5)
    single.step(1e-13, 5)
    torch.cuda.synchronize()
    for f in range(2):
        assert torch.equal(B.get_m(1, f), single.get_m(f)), f
        assert not torch.equal(B.get_m(0, f), single.get_m(f)), f   # instance 0 has no field
    B.close()
    single.close()


def test_validation():
    import paper_1801_04181_amd as mmv
    from workloads import get_config
    d, m = films(32)
    mesh = mmv.Mesh(d, Drive(), m)
    with pytest.raises(mmv.MMVError) as e:
        mmv.set_hext_field(mesh.h, 2, None)
    assert e.value.code == -1
    mesh.close()
    cube = get_config("cube_eddy")["desc"].replace(nx=8, ny=8, nz=8)
    c = mmv.Mesh(cube, Drive())
    with pytest.raises(mmv.MMVError) as e:
        mmv.set_hext_field(c.h, 0, None)
    assert e.value.code == -6
    c.close()
