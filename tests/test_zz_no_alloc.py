"""stray_force_noalloc (the entry point for callers that cannot allocate:
static device scratch, no synchronisation) against stray_force, which runs
the same kernels with the mesh's own partial-sum buffers: equal bit for bit,
and within the force bar of the float64 oracle.  Two calls in a row, the
second on a smaller mesh, so the second reuses the first one's scratch."""
import numpy as np
import pytest

from workloads import Desc, Drive
from workloads.states import domain_state
from gpu_common import oracle_system

pytestmark = pytest.mark.gpu

TOL_F = {32: 1e-5, 64: 1e-9}   # the force bars of the field tests


def films(prec, nx, ny, seed):
    d = Desc(n_films=2, nx=nx, ny=ny, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=1,
             max_travel_cells=3, Ms=1.1e6, Aex=1.5e-11, alpha=0.1, Ku=8e5, precision=prec)
    m = [domain_state((1, ny, nx), seed), domain_state((1, ny, nx), seed + 1)]
    return d, m


@pytest.mark.parametrize("prec", [32, 64])
def test_noalloc_force_equals_stray_force(prec):
    import torch
    import paper_1801_04181_amd as mmv
    for nx, ny, x_cells, seed in ((96, 40, 1.37, 41), (24, 9, -0.6, 43)):
        print(f"noalloc force fp{prec} {nx}x{ny} x={x_cells}", flush=True)
        d, m = films(prec, nx, ny, seed)
        mesh = mmv.Mesh(d, Drive(), m)
        mesh.set_offset(x_cells)
        F_dev = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda:0")
        mmv.stray_force_noalloc(mesh.h, F_dev)
        torch.cuda.synchronize()
        got = F_dev.cpu().numpy()
        ref = np.array(mesh.force())
        print("  noalloc", got, "stray_force", ref, flush=True)
        assert np.array_equal(got, ref)
        s = oracle_system(d, Drive(), m, x_cells)
        F_or = s.force()
        assert np.linalg.norm(got - F_or) <= TOL_F[prec] * np.linalg.norm(F_or)
        mesh.close()


def test_noalloc_force_after_steps_and_in_a_graph():
    """After spring-driven steps, and recorded into a HIP graph (no
    allocation during capture): every replay equals stray_force."""
    import torch
    import paper_1801_04181_amd as mmv
    from workloads import slider_mass_damping
    d, m = films(32, 64, 24, 47)
    mass, gv = slider_mass_damping(64, 24, 1e-3)
    drv = Drive(mode=2, v_d=5.0, k=1e-3, mass=mass, gamma_v=gv, x0=0.4 * d.dx)
    st = torch.cuda.Stream()
    mesh = mmv.Mesh(d, drv, m, stream=st)
    F_dev = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    with torch.cuda.stream(st):
        g = torch.cuda.CUDAGraph()
        mesh.step(1e-13, 5)
        st.synchronize()
        g.capture_begin()
        mmv.stray_force_noalloc(mesh.h, F_dev)
        g.capture_end()
        for rep in range(3):
            mesh.step(1e-13, 5)
            g.replay()
            st.synchronize()
            got = F_dev.cpu().numpy().copy()
            ref = np.array(mesh.force())
            print(f"  replay {rep}: noalloc {got} stray_force {ref}", flush=True)
            assert np.array_equal(got, ref)
    mesh.close()
