"""GPU parity: the HIP path through the C ABI vs the float64 oracle."""
import math
import numpy as np
import pytest

from workloads import Desc, Drive, get_config, initial_state
from workloads.states import random_unit, domain_state
from gpu_common import TERMS, TOL, TOL_CROSS, rel, max_rel, oracle_system

pytestmark = pytest.mark.gpu


def _mmv():
    import paper_1801_04181_amd as mmv
    return mmv


def check_fields(desc, drive, m, x_cells=None, tol=None):
    mmv = _mmv()
    tol_cross = tol or TOL_CROSS[desc.precision]
    tol = tol or TOL[desc.precision]
    print(f"fields: n_films={desc.n_films} {desc.nx}x{desc.ny} p{desc.precision} x={x_cells}", flush=True)
    mesh = mmv.Mesh(desc, drive, m)
    if x_cells is not None:
        mesh.set_offset(x_cells)
    s = oracle_system(desc, drive, m, x_cells)
    terms, F = s.field_terms()
    worst = {}
    for f in range(desc.n_films):
        for name, bit in TERMS:
            ref = terms[f][name]
            got = mesh.eval_heff(f, bit).cpu().numpy()
            if not np.any(ref):
                assert np.abs(got).max() == 0.0, (f, name)
                continue
            worst[(f, name)] = rel(got, ref)
            worst[(f, name, "max")] = max_rel(got, ref)
        tot = sum(terms[f][k] for k, _ in TERMS)
        worst[(f, "total")] = rel(mesh.eval_heff(f, 63).cpu().numpy(), tot)
    if desc.n_films == 2:
        Fg = np.array(mesh.force())
        worst["force"] = np.linalg.norm(Fg - F) / np.linalg.norm(F)
        print(f"  force gpu {Fg} oracle {F}", flush=True)
    mesh.close()
    print("  errors", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    for k, e in worst.items():
        cross = k == "force" or "demag_cross" in k
        assert e <= (tol_cross if cross else tol), (k, e)
    return worst


def test_tiny_fp64_fields():
    cfg = get_config("tiny")
    check_fields(cfg["desc"], cfg["drive"], initial_state(cfg), x_cells=0.37)


@pytest.mark.parametrize("x_cells", [0.37, 3.6, -2.25, 4.0, -4.0])
def test_stickslip_fp32_fields_full_size(x_cells):
    cfg = get_config("stickslip")
    check_fields(cfg["desc"], cfg["drive"], initial_state(cfg), x_cells=x_cells)


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("shape", [(60, 64), (128, 128), (256, 256)])
def test_compiled_fft_lengths(prec, shape):
    # transform lengths with compile-time plans (radices 5 6 9 / 6 3 4 / 5 9 3 /
    # 7 5 4 / 7 5 5 3): x 144, 280, 540 (half lengths 72, 140, 270), y 135,
    # 270, 525 -- odd, half-table and full-table twiddle variants
    import paper_1801_04181_amd as mmv
    nx, ny = shape
    cfg = get_config("stickslip")
    d = cfg["desc"].replace(nx=nx, ny=ny, precision=prec)
    h = mmv.init_mesh(d)
    lx, ly, _ = mmv.get_fft_lengths(h)
    mmv.destroy_mesh(h)
    assert (lx // 2, ly) in {(72, 135), (140, 270), (270, 525)}
    print("compiled lengths", nx, ny, lx, ly, prec, flush=True)
    check_fields(d, cfg["drive"], initial_state(dict(cfg, desc=d)), x_cells=1.37)


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("shape", [(37, 23), (5, 1), (1, 6), (70, 3)])
def test_ragged_shapes(prec, shape):
    nx, ny = shape
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=3e-9, dz=2.5e-9, gap_cells=2,
             max_travel_cells=3, Ms=9e5, Aex=1.2e-11, alpha=0.2, Ku=3e5, u=(0.3, -0.2, 0.9),
             Hext=(1e4, -2e4, 5e3), precision=prec)
    rng = np.random.default_rng(nx * 100 + ny)
    m = [random_unit((1, ny, nx), rng) for _ in range(2)]
    check_fields(d, Drive(), m, x_cells=1.3)
    check_fields(d, Drive(), m, x_cells=-2.9)


@pytest.mark.parametrize("prec", [32, 64])
def test_gap_zero_and_single_film(prec):
    d = Desc(n_films=2, nx=24, ny=17, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=0,
             max_travel_cells=2, Ms=1.1e6, Aex=1.5e-11, alpha=0.1, Ku=8e5, precision=prec)
    m = [domain_state((1, 17, 24), 3), domain_state((1, 17, 24), 4)]
    check_fields(d, Drive(), m, x_cells=0.5)
    d1 = d.replace(n_films=1)
    check_fields(d1, Drive(), m[:1])


@pytest.mark.parametrize("prec,nx,ny", [(32, 1728, 8), (64, 844, 8), (32, 16, 809), (64, 16, 404)])
def test_largest_meshes(prec, nx, ny):
    """The largest two-film meshes init_mesh accepts with the default halo
    and travel (a film row, or a spectrum column, in one CU's LDS): every
    term and the force against the oracle."""
    d = get_config("stickslip")["desc"].replace(nx=nx, ny=ny, precision=prec)
    m = [domain_state((1, ny, nx), 11), domain_state((1, ny, nx), 12)]
    check_fields(d, Drive(), m, x_cells=1.7)


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("halo", [2, 64])
def test_halo_extremes(prec, halo):
    """The smallest and largest spline halo the descriptor accepts."""
    d = Desc(n_films=2, nx=40, ny=12, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=1, max_travel_cells=3,
             halo=halo, Ms=1.1e6, Aex=1.5e-11, alpha=0.1, Ku=8e5, precision=prec)
    m = [domain_state((1, 12, 40), 21), domain_state((1, 12, 40), 22)]
    check_fields(d, Drive(), m, x_cells=2.6)
    check_fields(d, Drive(), m, x_cells=-3.0)


def run_steps(desc, drive, m, dt, n):
    mmv = _mmv()
    import torch
    mesh = mmv.Mesh(desc, drive, m)
    s = oracle_system(desc, drive, m)
    mesh.step(dt, n)
    torch.cuda.synchronize()
    s.run(dt, n)
    st = mesh.state()
    dm = max(np.abs(mesh.get_m(f).cpu().numpy() - s.m[f]).max() for f in range(desc.n_films))
    mesh.close()
    return dm, st, s


def test_tiny_fp64_100_steps():
    cfg = get_config("tiny")
    dm, st, s = run_steps(cfg["desc"], cfg["drive"], initial_state(cfg), cfg["dt"], 100)
    print("tiny 100 steps max|dm|", dm, flush=True)
    assert st["step"] == 100
    assert st["t"] == pytest.approx(s.t, rel=1e-15)
    assert dm < 1e-9


def test_spring_fp32_steps():
    d = Desc(n_films=2, nx=96, ny=40, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=1,
             max_travel_cells=4, Ms=1.1e6, Aex=1.5e-11, alpha=0.1, Ku=8e5, precision=32)
    from workloads import slider_mass_damping
    mass, gv = slider_mass_damping(96, 40, 1e-3)
    drv = Drive(mode=2, v_d=5.0, k=1e-3, mass=mass, gamma_v=gv, x0=0.9 * 2e-9)
    m = [domain_state((1, 40, 96), 7), domain_state((1, 40, 96), 8)]
    dm, st, s = run_steps(d, drv, m, 1e-13, 60)
    print("spring 60 steps max|dm|", dm, "x gpu", st["x"], "oracle", s.x, flush=True)
    assert dm < 1e-4
    assert abs(st["x"] - s.x) < 1e-4 * d.dx
    assert abs(st["v"] - s.v) < 1e-4 * max(abs(s.v), 1e-3)


# ---------------------------------------------------------------- scalar potential mode
@pytest.mark.parametrize("prec,nx,ny", [(32, 944, 16), (64, 459, 16), (32, 32, 781), (64, 32, 402)])
def test_largest_potential_meshes(prec, nx, ny):
    """The largest meshes init_mesh accepts in the scalar-potential mode
    (gap 3, halo 4; more rows per task than the direct mode)."""
    d = get_config("tiny_potential")["desc"].replace(nx=nx, ny=ny, precision=prec)
    m = [domain_state((1, ny, nx), 11), domain_state((1, ny, nx), 12)]
    check_fields(d, Drive(), m, x_cells=0.0)


def test_largest_mesh_spring_steps():
    """Three RK4 steps with the spring drive on the widest float32 mesh."""
    from workloads import slider_mass_damping
    nx, ny = 1728, 8
    d = get_config("stickslip")["desc"].replace(nx=nx, ny=ny, precision=32)
    mass, gv = slider_mass_damping(nx, ny, 1e-3)
    drv = Drive(mode=2, v_d=5.0, k=1e-3, mass=mass, gamma_v=gv, x0=0.6 * d.dx)
    m = [domain_state((1, ny, nx), 13), domain_state((1, ny, nx), 14)]
    dm, st, s = run_steps(d, drv, m, 1e-13, 3)
    print("largest mesh 3 steps max|dm|", dm, "x gpu", st["x"], "oracle", s.x, flush=True)
    assert dm < 1e-4
    assert abs(st["x"] - s.x) < 1e-4 * d.dx


def test_tiny_potential_fp64_fields():
    cfg = get_config("tiny_potential")
    check_fields(cfg["desc"], cfg["drive"], initial_state(cfg), x_cells=0.37)
    check_fields(cfg["desc"].replace(max_travel_cells=2), cfg["drive"], initial_state(cfg),
                 x_cells=-1.6)


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("shape", [(37, 23), (6, 2)])
def test_potential_ragged(prec, shape):
    nx, ny = shape
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=3e-9, dz=2.5e-9, gap_cells=3,
             max_travel_cells=3, Ms=9e5, Aex=1.2e-11, alpha=0.2, Ku=3e5, u=(0.3, -0.2, 0.9),
             precision=prec, cross_mode=1)
    rng = np.random.default_rng(nx + 7 * ny)
    m = [random_unit((1, ny, nx), rng) for _ in range(2)]
    check_fields(d, Drive(), m, x_cells=1.3)


def test_tiny_potential_fp64_100_steps():
    cfg = get_config("tiny_potential")
    dm, st, s = run_steps(cfg["desc"], cfg["drive"], initial_state(cfg), cfg["dt"], 100)
    print("tiny potential 100 steps max|dm|", dm, flush=True)
    assert dm < 1e-9


def test_profile_repeat_times_each_kernel_and_validates():
    import paper_1801_04181_amd as mmv
    cfg = get_config("tiny")
    d = cfg["desc"].replace(precision=32)
    mesh = mmv.Mesh(d, cfg["drive"], initial_state(cfg))
    for k in ("row_fwd", "col", "row_stage"):
        ms = mmv.profile_repeat(mesh.h, k, 5)
        assert 0.0 < ms < 100.0, (k, ms)
    for bad in (0, 4):
        with pytest.raises(mmv.MMVError) as e:
            mmv.profile_repeat(mesh.h, bad, 5)
        assert e.value.code == -1
    with pytest.raises(mmv.MMVError):
        mmv.profile_repeat(mesh.h, 2, 0)
    single = mmv.Mesh(d.replace(n_films=1), cfg["drive"])
    with pytest.raises(mmv.MMVError) as e:
        mmv.profile_repeat(single.h, 2, 5)
    assert e.value.code == -6
