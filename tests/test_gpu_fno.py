"""Learned stray-field operator on the GPU against the float64 reference
network: the BF16 matrix-core product on its own (lane layout, strides,
ragged tiles), then forward values, loss, gradients and one Adam step.

Bars.  The product rounds both operands to bfloat16 (relative 2^-9) and
accumulates in float32, so against float64 of the *rounded* operands it is
exact to float32 summation error: 1e-5 of the output's scale.  Through the
network every product rounds its operands; rounding errors of 2^-9 per
operand add in quadrature over ~20 chained products per output, giving
~1e-2 relative-L2 on the outputs and ~3e-2 on the gradients (observed
3-5x below these bars).
"""
import numpy as np
import pytest
import torch

from oracle import fno
from workloads.fno_inputs import init_params, operator_inputs

pytestmark = pytest.mark.gpu


def bf16(x):
    return torch.as_tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("M,N,K,ta,tb,tc", [
    (32, 32, 8, False, False, False),      # one MFMA tile, one k step
    (64, 64, 64, False, False, False),
    (70, 100, 45, False, False, False),    # ragged in every dimension
    (70, 100, 45, True, True, False),      # transposed operands
    (33, 65, 129, False, True, True),      # transposed output
    (200, 17, 300, False, True, False),    # narrow N: 128 x 32 block tiles
    (20, 150, 70, True, False, True),      # narrow M: 32 x 128 block tiles
    (32, 16, 256, True, False, False),     # small product, k steps split over the waves
    (20, 30, 300, False, True, True),      # small, ragged, three k chunks
    (1, 1, 1, False, False, False)])
def test_gemm_matches_float64_of_rounded_operands(M, N, K, ta, tb, tc):
    import paper_1801_04181_amd as mmv
    print("gemm", M, N, K, ta, tb, tc, flush=True)
    g = torch.Generator().manual_seed(M * 1000 + N * 10 + K)
    A = torch.randn(M, K, generator=g, dtype=torch.float32)
    B = torch.randn(K, N, generator=g, dtype=torch.float32)
    C0 = torch.randn(M, N, generator=g, dtype=torch.float32)
    Ad = (A.t().contiguous() if ta else A).cuda()
    Bd = (B.t().contiguous() if tb else B).cuda()
    Cd = (C0.t().contiguous() if tc else C0).cuda()
    am, ak = (1, M) if ta else (K, 1)
    bk, bn = (1, K) if tb else (N, 1)
    cm, cn = (1, M) if tc else (N, 1)
    mmv.sur_gemm_bf16(Ad, am, ak, Bd, bk, bn, Cd, cm, cn, M, N, K, 0.75, -0.5)
    torch.cuda.synchronize()
    out = Cd.cpu().double()
    out = out.t() if tc else out
    ref = 0.75 * (bf16(A) @ bf16(B)) - 0.5 * C0.double()
    scale = float((bf16(A).abs() @ bf16(B).abs()).max()) + 1.0
    assert float((out - ref).abs().max()) <= 1e-5 * scale


def _net(H, W, C, Mx, My, L, B, seed):
    import paper_1801_04181_amd as mmv
    s = mmv.Surrogate(H, W, C, Mx, My, L, max_batch=B)
    w = init_params(C, Mx, My, L, seed, bias_scale=0.1)
    # larger spectral weights than the initial scale, so that the spectral
    # path carries a share of the output comparable to the pointwise path
    lay, n = fno.layout(C, Mx, My, L)
    for l in range(L):
        o, shp = lay[f"R{l}"]
        w[o:o + int(np.prod(shp))] *= 40.0
    assert s.n == n
    s.set_params(torch.from_numpy(w).float())
    return s, torch.from_numpy(w).float().double()


def test_parameter_offsets_match_the_reference_layout():
    import paper_1801_04181_amd as mmv
    for C, Mx, My, L in [(32, 16, 32, 4), (5, 3, 6, 2)]:
        s = mmv.Surrogate(64, 48, C, Mx, My, L, max_batch=1)
        lay, n = fno.layout(C, Mx, My, L)
        names = ["wl", "bl"] + [f"{k}{l}" for l in range(L) for k in ("R", "wp", "bp")] + ["wq", "bq"]
        assert s.n == n
        assert s.offsets == [lay[k][0] for k in names]
        s.close()


CASES = [
    # H, W, C, Mx, My, L, B: several tiles with ragged tails; the full-size network
    (40, 36, 8, 5, 6, 2, 3),
    (64, 64, 32, 16, 32, 4, 2),
    (256, 256, 32, 16, 32, 4, 2),
]


@pytest.mark.parametrize("H,W,C,Mx,My,L,B", CASES)
def test_forward_loss_and_gradient_match_reference(H, W, C, Mx, My, L, B):
    print("fno", H, W, C, Mx, My, L, B, flush=True)
    s, w = _net(H, W, C, Mx, My, L, B, seed=H + C)
    a = torch.from_numpy(operator_inputs(B, H, W, seed=7 + H))
    t = torch.from_numpy(np.random.default_rng(8).standard_normal((B, 3, H, W)) * 0.5)
    ad, td = a.float().cuda(), t.float().cuda()
    out = s.forward(ad).cpu().double()
    ref = fno.forward(w, a, C, Mx, My, L)
    assert rel(out, ref) < 1e-2
    loss, g = s.gradient(ad, td)
    torch.cuda.synchronize()
    lref, gref = fno.loss_and_grad(w, a, t, C, Mx, My, L)
    assert abs(loss - lref) <= 2e-2 * lref
    g = g.cpu().double()
    assert rel(g, gref) < 3e-2
    lay, _ = fno.layout(C, Mx, My, L)
    for name, (o, shp) in lay.items():
        k = int(np.prod(shp))
        if float(gref[o:o + k].norm()) > 1e-3 * float(gref.norm()):
            assert rel(g[o:o + k], gref[o:o + k]) < 5e-2, name
    s.close()


def test_adam_step_moves_each_weight_by_lr_against_the_gradient_sign():
    H, W, C, Mx, My, L, B = 32, 32, 8, 4, 8, 2, 2
    s, w = _net(H, W, C, Mx, My, L, B, seed=11)
    a = torch.from_numpy(operator_inputs(B, H, W, seed=12))
    t = torch.from_numpy(np.random.default_rng(13).standard_normal((B, 3, H, W)))
    _, gref = fno.loss_and_grad(w, a, t, C, Mx, My, L)
    w0 = s.get_params().cpu().double()
    lr = 1e-3
    loss, relerr = s.train_step(a.float().cuda(), t.float().cuda(), lr)
    torch.cuda.synchronize()
    dw = s.get_params().cpu().double() - w0
    # first bias-corrected step: dw = -lr g / (|g| + 1e-8), i.e. -lr sign(g)
    # wherever |g| is far above the gradient's rounding noise
    noise = 0.05 * float(gref.abs().max())
    sure = gref.abs() > noise
    assert int(sure.sum()) > 100
    assert torch.allclose(dw[sure], -lr * torch.sign(gref[sure]), rtol=0, atol=lr * 1e-3)
    assert float(dw.abs().max()) <= lr * (1 + 1e-3)
    lref = float(fno.loss(w, a, t, C, Mx, My, L))
    assert abs(loss - lref) <= 2e-2 * lref
    assert 0 < relerr < 10
    s.close()


def test_training_reduces_the_loss_on_a_fixed_batch():
    H, W, C, Mx, My, L, B = 32, 32, 8, 4, 8, 2, 4
    s, w = _net(H, W, C, Mx, My, L, B, seed=21)
    a = torch.from_numpy(operator_inputs(B, H, W, seed=22))
    # target: a smooth linear functional of the input, reachable by the network
    t = torch.stack([a[:, 2] * 0.3, a[:, 0] - a[:, 1], 0.5 * a[:, 2].roll(3, dims=-1)], dim=1)
    ad, td = a.float().cuda(), t.float().cuda()
    first = None
    for k in range(150):
        loss, _ = s.train_step(ad, td, 3e-3)
        first = loss if first is None else first
    final = s.gradient(ad, td)[0]
    assert np.isfinite(final) and final < 0.2 * first
    s.close()
