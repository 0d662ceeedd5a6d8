"""Seeded inputs of the learned stray-field operator.

Random draws only: initial parameter vectors and network inputs.  The
caller passes the parameter blocks (start offset, element count, fan-in
scale); nothing here knows the network's arithmetic.
"""
import numpy as np

from .states import domain_state


def param_blocks(C, Mx, My, L):
    """(name, count, scale) per parameter block in storage order, with
    uniform(-scale, scale) initialisation: fan-in scaling for the pointwise
    weights, 1/C^2 for the spectral weights, zero biases."""
    P = Mx * My
    b = [("wl", 4 * C, 0.5), ("bl", C, 0.0)]
    for l in range(L):
        b += [(f"R{l}", 2 * P * C * C, 1.0 / (C * C)), (f"wp{l}", C * C, C ** -0.5),
              (f"bp{l}", C, 0.0)]
    b += [("wq", 3 * C, C ** -0.5), ("bq", 3, 0.0)]
    return b


def init_params(C, Mx, My, L, seed, bias_scale=0.0):
    """float64 vector of the concatenated blocks; biases uniform(+-bias_scale)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, n, scale in param_blocks(C, Mx, My, L):
        if name[0] == "b":
            scale = bias_scale
        parts.append(scale * (2.0 * rng.random(n) - 1.0))
    return np.concatenate(parts)


def operator_inputs(B, H, W, seed, travel_cells=4.0, state="domains"):
    """[B][4][H][W] float64: slider magnetisation (3 channels) and its offset
    in cells x_p (uniform in [0, travel_cells]) broadcast as the 4th channel."""
    rng = np.random.default_rng(seed)
    a = np.empty((B, 4, H, W))
    for b in range(B):
        s = int(rng.integers(1 << 30))
        if state == "domains":
            a[b, :3] = domain_state((1, H, W), s)[:, 0]
        else:
            m = np.random.default_rng(s).standard_normal((3, H, W))
            a[b, :3] = m / np.sqrt((m * m).sum(axis=0, keepdims=True))
        a[b, 3] = rng.uniform(0.0, travel_cells)
    return a
