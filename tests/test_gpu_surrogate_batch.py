"""The learned operator inside batched steps (the surrogate + batched form):
one batched inference per RK stage over every instance replaces film 0's
cross field.  Each instance must follow the same trajectory as the same
mesh stepped alone with the operator attached (itself checked against the
float64 reference composition in test_gpu_surrogate.py); the batch-wide
error judge and its fallback to the exact path; attach-time validation."""
import numpy as np
import pytest
import torch

from workloads import get_config, initial_state, Drive, slider_mass_damping
from workloads.fno_inputs import init_params
from workloads.states import domain_state
from oracle import fno

pytestmark = pytest.mark.gpu

C, MX, MY, L = 8, 5, 6, 2


def setup(n=3, nx=40, ny=48, scale=1.0):
    cfg = get_config("learned")
    d = cfg["desc"].replace(nx=nx, ny=ny)
    w = init_params(C, MX, MY, L, seed=3, bias_scale=0.1)
    lay, _ = fno.layout(C, MX, MY, L)
    for l in range(L):
        o, shp = lay[f"R{l}"]
        w[o:o + int(np.prod(shp))] *= 40.0
    w = (w * scale).astype(np.float32)
    ms, drives = [], []
    mass, gv = slider_mass_damping(nx, ny, 1e-3)
    for i in range(n):
        ms.append([domain_state((1, ny, nx), 70 + 2 * i), domain_state((1, ny, nx), 71 + 2 * i)])
        drives.append(Drive(mode=2, v_d=1.0 + i, k=1e-3, mass=mass, gamma_v=gv, x0=0.2 * i * d.dx))
    return cfg, d, ms, drives, w


def test_batched_operator_equals_single_meshes():
    import paper_1801_04181_amd as mmv
    cfg, d, ms, drives, w = setup()
    n = len(ms)
    print("batched surrogate", n, d.nx, d.ny, flush=True)
    s = mmv.Surrogate(d.ny, d.nx, C, MX, MY, L, max_batch=n)
    s.set_params(torch.from_numpy(w))
    B = mmv.Batch([d] * n, drives, ms)
    mmv.batch_sur_attach(B.b, s.h, 1000, 1e9)
    B.step(cfg["dt"], 3)
    torch.cuda.synchronize()
    err, fell, judged = mmv.batch_sur_status(B.b)
    assert judged == 1 and not fell and err > 0
    worst = 0.0
    for i in range(n):
        M = mmv.Mesh(d, drives[i], ms[i])
        mmv.sur_attach(M.h, s.h, 1000, 1e9)
        M.step(cfg["dt"], 3)
        torch.cuda.synchronize()
        for f in range(2):
            a = B.get_m(i, f).cpu().numpy()
            b = M.get_m(f).cpu().numpy()
            worst = max(worst, np.abs(a - b).max())
        sb, s1 = B.state(i), M.state()
        assert sb["step"] == s1["step"] == 3
        assert abs(sb["x"] - s1["x"]) <= 1e-9 * d.dx
        M.close()
    print("  max |dm| batch vs single", worst, flush=True)
    assert worst <= 1e-6
    B.close()


@pytest.mark.parametrize("tol,fallback", [(0.5, True), (2.0, False)])
def test_batch_judge_and_fallback(tol, fallback):
    import paper_1801_04181_amd as mmv
    cfg, d, ms, drives, w = setup(n=2, scale=0.0)   # zero network: error exactly 1
    s = mmv.Surrogate(d.ny, d.nx, C, MX, MY, L, max_batch=2)
    s.set_params(torch.from_numpy(w))
    B = mmv.Batch([d] * 2, drives, ms)
    P = mmv.Batch([d] * 2, drives, ms)
    mmv.batch_sur_attach(B.b, s.h, 2, tol)
    B.step(cfg["dt"], 5)
    P.step(cfg["dt"], 5)
    torch.cuda.synchronize()
    err, fell, judged = mmv.batch_sur_status(B.b)
    assert abs(err - 1.0) < 1e-6
    assert fell == fallback
    assert judged == (1 if fallback else 3)
    for i in range(2):
        a = B.get_m(i, 0).cpu().numpy()
        b = P.get_m(i, 0).cpu().numpy()
        if fallback:
            assert np.array_equal(a, b) and B.state(i) == P.state(i)
        else:
            assert not np.array_equal(a, b)
    B.close()
    P.close()


def test_batch_attach_validation():
    import paper_1801_04181_amd as mmv
    cfg, d, ms, drives, w = setup(n=3)
    B = mmv.Batch([d] * 3, drives, ms)
    small = mmv.Surrogate(d.ny, d.nx, C, MX, MY, L, max_batch=2)
    with pytest.raises(mmv.MMVError) as e:
        mmv.batch_sur_attach(B.b, small.h, 10, 1e-3)
    assert e.value.code == -1
    other = mmv.Surrogate(d.ny + 2, d.nx, C, MX, MY, L, max_batch=4)
    with pytest.raises(mmv.MMVError) as e:
        mmv.batch_sur_attach(B.b, other.h, 10, 1e-3)
    assert e.value.code == -1
    B.close()
    d64 = d.replace(precision=64)
    B64 = mmv.Batch([d64], drives[:1], ms[:1])
    ok = mmv.Surrogate(d.ny, d.nx, C, MX, MY, L, max_batch=1)
    with pytest.raises(mmv.MMVError) as e:
        mmv.batch_sur_attach(B64.b, ok.h, 10, 1e-3)
    assert e.value.code == -6
    B64.close()
