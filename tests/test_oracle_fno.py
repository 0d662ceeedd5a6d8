"""Pins of the reference learned operator (oracle/fno.py) against facts
fixed by the mathematics: band-limited identity, a plane wave through one
complex weight, the per-pixel MLP it reduces to without spectral weights,
central differences for the gradient, the erf GELU, a worked Adam step."""
import math
import numpy as np
import pytest
import torch

from oracle import fno
from workloads.fno_inputs import init_params, operator_inputs, param_blocks


def _identity_R(C, Mx, My):
    R = torch.zeros(Mx * My, 2, C, C, dtype=torch.float64)
    R[:, 0] = torch.eye(C, dtype=torch.float64)
    return R


def test_layout_total_closed_form():
    for C, Mx, My, L in [(32, 16, 32, 4), (3, 2, 4, 1), (8, 5, 6, 3)]:
        lay, n = fno.layout(C, Mx, My, L)
        assert n == 5 * C + L * (2 * Mx * My * C * C + C * C + C) + 3 * C + 3
        assert n == sum(k for _, k, _ in param_blocks(C, Mx, My, L))
        assert lay["wq"][0] == n - 3 * C - 3


def test_identity_weights_reproduce_band_limited_field():
    H, W, C, Mx, My = 16, 20, 2, 4, 6
    rng = np.random.default_rng(0)
    X = np.zeros((1, C, H, W // 2 + 1), dtype=complex)
    for ky in list(range(My // 2)) + list(range(H - My // 2 + 1, H)):
        for kx in range(Mx):
            X[0, :, ky, kx] = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    v = torch.fft.irfft2(torch.from_numpy(X), s=(H, W))
    out = fno.spectral_conv(v, _identity_R(C, Mx, My), Mx, My)
    assert torch.allclose(out, v, atol=1e-13 * float(v.abs().max()))


def test_identity_weights_drop_modes_outside_the_kept_set():
    H, W, C, Mx, My = 16, 16, 1, 3, 4
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    v = torch.from_numpy(np.cos(2 * np.pi * (Mx * xx / W + yy / H)))[None, None]
    out = fno.spectral_conv(v, _identity_R(C, Mx, My), Mx, My)
    assert float(out.abs().max()) < 1e-13


@pytest.mark.parametrize("kx,ky_slot", [(1, 1), (2, 5), (0, 6), (3, 0)])
def test_plane_wave_through_one_complex_weight(kx, ky_slot):
    H, W, Mx, My = 16, 12, 4, 8
    ky = fno.ky_of_slot(H, My)[ky_slot]
    cr, ci = 0.7, -1.3
    R = torch.zeros(Mx * My, 2, 1, 1, dtype=torch.float64)
    R[ky_slot * Mx + kx, 0] = cr
    R[ky_slot * Mx + kx, 1] = ci
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    th = 2 * np.pi * (kx * xx / W + ky * yy / H)
    v = torch.from_numpy(np.cos(th))[None, None]
    out = fno.spectral_conv(v, R, Mx, My)[0, 0].numpy()
    if kx == 0:
        # a real cosine along y has both +ky and -ky; only slot ky is kept, so
        # half its amplitude passes, and the real part is taken
        expect = 0.5 * (cr * np.cos(th) - ci * np.sin(th))
    else:
        expect = cr * np.cos(th) - ci * np.sin(th)
    assert np.abs(out - expect).max() < 1e-12


def test_without_spectral_weights_the_network_is_a_per_pixel_mlp():
    C, Mx, My, L, H, W = 3, 2, 2, 2, 4, 5
    w = torch.from_numpy(init_params(C, Mx, My, L, seed=1, bias_scale=0.3))
    p = fno.unpack(w, C, Mx, My, L)
    for l in range(L):
        p[f"R{l}"].zero_()
    a = torch.from_numpy(operator_inputs(2, H, W, seed=2, state="random"))
    out = fno.forward(w, a, C, Mx, My, L).numpy()
    P = {k: v.numpy() for k, v in p.items()}

    def g(x):
        return 0.5 * x * (1 + math.erf(x / math.sqrt(2)))  # erf form, 1e-3 off tanh form

    for b in range(2):
        for y in range(H):
            for x in range(W):
                v = [sum(P["wl"][c][j] * a[b, j, y, x].item() for j in range(4)) + P["bl"][c]
                     for c in range(C)]
                for l in range(L):
                    pre = [sum(P[f"wp{l}"][o][i] * v[i] for i in range(C)) + P[f"bp{l}"][o]
                           for o in range(C)]
                    v = [0.5 * t * (1 + math.tanh(math.sqrt(2 / math.pi) * (t + 0.044715 * t ** 3)))
                         for t in pre]
                    assert all(abs(vt - g(t)) < 1e-3 for vt, t in zip(v, pre))
                for o in range(3):
                    ref = sum(P["wq"][o][i] * v[i] for i in range(C)) + P["bq"][o]
                    assert abs(out[b, o, y, x] - ref) < 1e-12


def test_gelu_matches_tanh_gelu_and_erf_gelu():
    x = torch.linspace(-6, 6, 2001, dtype=torch.float64)
    assert torch.allclose(fno.gelu(x), torch.nn.functional.gelu(x, approximate="tanh"), atol=1e-15)
    erf = 0.5 * x * (1 + torch.erf(x / math.sqrt(2)))
    assert float((fno.gelu(x) - erf).abs().max()) < 1e-3


def test_gradient_matches_central_differences():
    C, Mx, My, L, H, W = 2, 2, 4, 2, 8, 8
    w = torch.from_numpy(init_params(C, Mx, My, L, seed=3, bias_scale=0.2))
    a = torch.from_numpy(operator_inputs(2, H, W, seed=4))
    t = torch.from_numpy(np.random.default_rng(5).standard_normal((2, 3, H, W)))
    _, g = fno.loss_and_grad(w, a, t, C, Mx, My, L)
    rng = np.random.default_rng(6)
    idx = rng.choice(w.numel(), 40, replace=False)
    lay, _ = fno.layout(C, Mx, My, L)
    idx = np.concatenate([idx, [o for o, _ in lay.values()]])  # first entry of every block
    h = 1e-6
    for i in idx:
        wp, wm = w.clone(), w.clone()
        wp[i] += h
        wm[i] -= h
        fd = (float(fno.loss(wp, a, t, C, Mx, My, L)) - float(fno.loss(wm, a, t, C, Mx, My, L))) / (2 * h)
        assert abs(fd - float(g[i])) <= 1e-7 + 1e-5 * abs(fd), (i, fd, float(g[i]))


def test_adam_first_step_is_a_signed_lr_step():
    w = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64)
    g = torch.tensor([0.3, -1e-3, 5.0, 0.0], dtype=torch.float64)
    z = torch.zeros(4, dtype=torch.float64)
    w1, m1, m2 = fno.adam(w, g, z, z, step=1, lr=0.01)
    # m1 = 0.1 g, m2 = 0.001 g^2; corrected: g and g^2, so the step is lr g / (|g| + eps)
    expect = w - 0.01 * g / (g.abs() + 1e-8)
    assert torch.allclose(w1, expect, atol=1e-15)
    assert torch.allclose(m1, 0.1 * g) and torch.allclose(m2, 0.001 * g * g)
    # second step with the same gradient: still lr * g / (|g| + eps') per entry
    w2, _, _ = fno.adam(w1, g, m1, m2, step=2, lr=0.01)
    assert torch.allclose(w2 - w1, expect - w, atol=1e-12)
