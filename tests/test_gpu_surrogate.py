"""The learned operator inside the LLG step (film 0's cross field from the
network at every RK stage) against the reference composition: the float64
oracle System whose base-film cross field is the float64 reference network
evaluated on the stage's slider state.  And the error judge: exact error
value, fallback to the exact path, and attach-time validation.

Bar.  The network's BF16 operands give its output a ~1e-3 relative error;
over three steps of dt = 1e-13 s that moves film 0's magnetisation by
~3e-5 relative-L2 (CPU emulation of the same arithmetic: 2.7e-5).  Film 1
only feels it through the slider position: ~1e-7."""
import numpy as np
import pytest
import torch

from oracle import fno
from oracle.sim import System
from workloads import get_config, initial_state
from workloads.fno_inputs import init_params
from gpu_common import rel

pytestmark = pytest.mark.gpu

C, MX, MY, L = 8, 5, 6, 2


def _setup(scale=1.0, nx=40, ny=48, **desc_kw):
    cfg = get_config("learned")
    d = cfg["desc"].replace(nx=nx, ny=ny, **desc_kw)
    m = initial_state(dict(cfg, desc=d))
    w = init_params(C, MX, MY, L, seed=3, bias_scale=0.1)
    lay, _ = fno.layout(C, MX, MY, L)
    for l in range(L):
        o, shp = lay[f"R{l}"]
        w[o:o + int(np.prod(shp))] *= 40.0
    w = (w * scale).astype(np.float32)
    return cfg, d, m, w


def _mesh(mmv, d, drive, m):
    return mmv.Mesh(d, drive, m)


def test_surrogate_step_matches_reference_composition():
    import paper_1801_04181_amd as mmv
    cfg, d, m, w = _setup()
    print("surrogate step", d.nx, d.ny, flush=True)
    s = mmv.Surrogate(d.ny, d.nx, C, MX, MY, L, max_batch=1)
    s.set_params(torch.from_numpy(w))
    M = _mesh(mmv, d, cfg["drive"], m)
    mmv.sur_attach(M.h, s.h, 1000, 1e9)
    M.step(cfg["dt"], 3)
    got = [M.get_m(f).cpu().numpy() for f in range(2)]
    st = M.state()
    err, fell, judged = mmv.sur_status(M.h)
    assert judged == 1 and not fell and err > 0

    ref = System(d, cfg["drive"], m)
    w64 = torch.from_numpy(w.astype(np.float64))

    def base_cross(ms, x):
        a = np.empty((1, 4, d.ny, d.nx))
        a[0, :3] = ms[:, 0]
        a[0, 3] = x / d.dx
        return d.Ms * fno.forward(w64, torch.from_numpy(a), C, MX, MY, L)[0].numpy()[:, None]

    ref.base_cross = base_cross
    ref.run(cfg["dt"], 3)
    assert rel(got[0], ref.m[0]) < 1e-4
    assert rel(got[1], ref.m[1]) < 1e-6
    assert abs(st["x"] - ref.x) <= 1e-4 * abs(ref.x)
    assert abs(st["v"] - ref.v) <= 1e-4 * abs(ref.v)


@pytest.mark.parametrize("tol,fallback", [(0.5, True), (2.0, False)])
def test_judge_error_and_fallback(tol, fallback):
    import paper_1801_04181_amd as mmv
    cfg, d, m, w = _setup(scale=0.0)      # network output is zero: error exactly 1
    print("judge", tol, flush=True)
    s = mmv.Surrogate(d.ny, d.nx, C, MX, MY, L, max_batch=1)
    s.set_params(torch.from_numpy(w))
    M = _mesh(mmv, d, cfg["drive"], m)
    plain = _mesh(mmv, d, cfg["drive"], m)
    mmv.sur_attach(M.h, s.h, 2, tol)
    M.step(cfg["dt"], 5)
    plain.step(cfg["dt"], 5)
    err, fell, judged = mmv.sur_status(M.h)
    assert abs(err - 1.0) < 1e-6
    assert fell == fallback
    assert judged == (1 if fallback else 3)     # steps 0, 2, 4
    a = [M.get_m(f).cpu().numpy() for f in range(2)]
    b = [plain.get_m(f).cpu().numpy() for f in range(2)]
    if fallback:                                # exact path from the first judge on
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
        assert M.state() == plain.state()
    else:                                       # film 0 ran without its cross field
        assert not np.array_equal(a[0], b[0])


def test_attach_validation():
    import paper_1801_04181_amd as mmv
    cfg, d, m, w = _setup()
    s = mmv.Surrogate(d.ny, d.nx, C, MX, MY, L, max_batch=1)
    for kw, code in [(dict(precision=64), -6), (dict(cross_mode=1, gap_cells=3), -6)]:
        M = mmv.Mesh(d.replace(**kw), cfg["drive"])
        with pytest.raises(mmv.MMVError) as e:
            mmv.sur_attach(M.h, s.h, 10, 1e-3)
        assert e.value.code == code
    M = mmv.Mesh(d.replace(nx=d.nx + 2), cfg["drive"])
    with pytest.raises(mmv.MMVError) as e:
        mmv.sur_attach(M.h, s.h, 10, 1e-3)
    assert e.value.code == -1
    M = mmv.Mesh(d, cfg["drive"])
    for every, tol in [(0, 1e-3), (10, 0.0), (10, float("nan"))]:
        with pytest.raises(mmv.MMVError):
            mmv.sur_attach(M.h, s.h, every, tol)
    mmv.sur_attach(M.h, s.h, 10, 1e-3)
    mmv.sur_attach(M.h, None, 10, 1e-3)      # detach
