"""Learned stray-field operator, reference form (float64, plain torch on CPU).

TEST INFRASTRUCTURE ONLY (see the package header).

The operator is a Fourier neural operator (Li et al., "Fourier neural
operator for parametric partial differential equations", ICLR 2021) that
stands in for the cross term of Eqs. (6)-(8) -- the slider's stray field on
the base film, sampled at the slider offset with the spline of Sec. III.A.
Its input per sample is [m_x, m_y, m_z, x_p] on the H x W base grid; its
output the three field components there.

  v_0     = W_l a + b_l                                   pointwise 4 -> C
  v_{l+1} = GELU( K_l v_l + W_p,l v_l + b_p,l )            l = 0 .. L-1
  K_l v   = irfft2( R_l(k) rfft2(v)(k) on the kept modes, zero elsewhere )
  out     = W_q v_L + b_q                                 pointwise C -> 3

kept modes: kx in [0, Mx) (half spectrum), ky in [0, My/2) and
[H - My/2, H); R_l(k) is a complex C x C matrix per kept mode.  GELU is the
tanh form, 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))).

Parameter vector (float): wl [C][4], bl [C], per layer R [P][2][C][C]
(mode p = ky_slot * Mx + kx, planes real / imaginary), Wp [C][C], bp [C];
then wq [3][C], bq [3].

Pins (tests/test_oracle_fno.py): identity spectral weights reproduce a
band-limited field; a single plane wave comes back multiplied by the complex
weight (sign and conjugation conventions); with R = 0 the network is a
per-pixel MLP, checked against an explicit per-pixel loop; the autograd
gradient against central differences; GELU against its erf form and torch's
own tanh GELU; Adam against a hand-worked first step.
"""
import math
import numpy as np
import torch


def layout(C, Mx, My, L):
    """Start offsets and shapes of every parameter block, and the total."""
    P = Mx * My
    blocks = [("wl", (C, 4)), ("bl", (C,))]
    for l in range(L):
        blocks += [(f"R{l}", (P, 2, C, C)), (f"wp{l}", (C, C)), (f"bp{l}", (C,))]
    blocks += [("wq", (3, C)), ("bq", (3,))]
    out, o = {}, 0
    for name, shape in blocks:
        out[name] = (o, shape)
        o += int(np.prod(shape))
    return out, o


def unpack(w, C, Mx, My, L):
    lay, n = layout(C, Mx, My, L)
    assert w.numel() == n
    return {k: w[o:o + int(np.prod(s))].view(*s) for k, (o, s) in lay.items()}


def gelu(x):
    return 0.5 * x * (1.0 + torch.tanh(math.sqrt(2.0 / math.pi) * (x + 0.044715 * x ** 3)))


def ky_of_slot(H, My):
    """Frequency index ky of each kept slot: 0 .. My/2-1, then H-My/2 .. H-1."""
    h = My // 2
    return [s if s < h else H - My + s for s in range(My)]


def spectral_conv(v, R, Mx, My):
    """K v for v [B][C][H][W] and R [P][2][C][C]; returns [B][C][H][W]."""
    B, C, H, W = v.shape
    X = torch.fft.rfft2(v)                                   # [B][C][H][W//2+1]
    Rc = torch.complex(R[:, 0], R[:, 1]).view(My, Mx, C, C)  # [ky_slot][kx][o][i]
    Y = torch.zeros_like(X)
    for s, ky in enumerate(ky_of_slot(H, My)):
        for kx in range(Mx):
            Y[:, :, ky, kx] = X[:, :, ky, kx] @ Rc[s, kx].T
    return torch.fft.irfft2(Y, s=(H, W))


def pointwise(wt, b, v):
    """wt [O][I] applied at every pixel of v [B][I][H][W], plus bias b [O]."""
    out = torch.einsum("oi,bihw->bohw", wt, v)
    return out + b.view(1, -1, 1, 1) if b is not None else out


def forward(w, a, C, Mx, My, L):
    """Network output [B][3][H][W] for parameters w and input a [B][4][H][W]."""
    p = unpack(w, C, Mx, My, L)
    v = pointwise(p["wl"], p["bl"], a)
    for l in range(L):
        v = gelu(spectral_conv(v, p[f"R{l}"], Mx, My) + pointwise(p[f"wp{l}"], p[f"bp{l}"], v))
    return pointwise(p["wq"], p["bq"], v)


def loss(w, a, t, C, Mx, My, L):
    """Mean over every output element of (out - t)^2."""
    return ((forward(w, a, C, Mx, My, L) - t) ** 2).mean()


def loss_and_grad(w, a, t, C, Mx, My, L):
    w = w.detach().clone().requires_grad_(True)
    val = loss(w, a, t, C, Mx, My, L)
    (g,) = torch.autograd.grad(val, w)
    return float(val.detach()), g.detach()


def adam(w, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma & Ba 2015); returns new w, m1, m2."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return w - lr * mh / (torch.sqrt(vh) + eps), m1, m2
