"""Training the learned stray-field operator on pairs from the exact path.

A pair is (input, target): the input holds the slider film's magnetisation
and its offset x_s / dx (channels m_x, m_y, m_z, x_p), the target the
slider's stray field on the base film -- the cross term of Eqs. (6)-(8)
sampled with the spline of Sec. III.A -- from eval_heff on film 0 with
only the cross bit set, divided by Ms.  Every pair is drawn fresh on the
GPU: a domain state from a seeded pool, rolled by a random lattice shift,
with m_z flipped at random, placed at a random offset in [0, travel].
"""
import math

import numpy as np

from . import Mesh, Surrogate, TERM, sur_attach, sur_status

__all__ = ["PairSource", "train", "held_out_error", "sur_attach", "sur_status"]


class PairSource:
    """Exact (input, target) pairs for a two-film mesh description."""

    def __init__(self, desc, pool, seed=0, device="cuda:0"):
        import torch
        self.torch = torch
        self.desc = desc
        self.dev = torch.device(device)
        self.mesh = Mesh(desc, device=device)
        self.pool = torch.as_tensor(np.asarray(pool), dtype=torch.float32).to(self.dev)  # [K][3][ny][nx]
        self.gen = np.random.default_rng(seed)
        self.travel = float(desc.max_travel_cells)

    def batch(self, B):
        torch = self.torch
        d = self.desc
        a = torch.empty((B, 4, d.ny, d.nx), dtype=torch.float32, device=self.dev)
        t = torch.empty((B, 3, d.ny, d.nx), dtype=torch.float32, device=self.dev)
        zero = torch.zeros((3, 1, d.ny, d.nx), dtype=torch.float32, device=self.dev)
        self.mesh.set_m(0, zero)
        for b in range(B):
            k = int(self.gen.integers(len(self.pool)))
            sy, sx = int(self.gen.integers(d.ny)), int(self.gen.integers(d.nx))
            m = torch.roll(self.pool[k], shifts=(sy, sx), dims=(-2, -1)).clone()
            if self.gen.random() < 0.5:
                m[2] = -m[2]
            x = float(self.gen.uniform(0.0, self.travel))
            self.mesh.set_m(1, m[:, None].contiguous())
            self.mesh.set_offset(x)
            h = self.mesh.eval_heff(0, TERM["demag_cross"])
            a[b, :3] = m
            a[b, 3] = x
            t[b] = h[:, 0] / d.Ms
        return a, t


def train(sur, source, steps, B=8, lr=2e-3, lr_final=1e-4, log=None, log_every=200):
    """Adam with a cosine learning-rate decay from lr to lr_final."""
    hist = []
    for k in range(steps):
        a, t = source.batch(B)
        r = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * k / max(1, steps - 1)))
        loss, rel = sur.train_step(a, t, r)
        if not math.isfinite(loss):
            raise FloatingPointError(f"training diverged at step {k}")
        hist.append(rel)
        if log is not None and (k % log_every == 0 or k == steps - 1):
            log(f"train step {k} lr {r:.2e} loss {loss:.4e} rel {rel:.4f}")
    return hist


def held_out_error(sur, source, n=32, B=8):
    """Relative L2 error ||net - exact|| / ||exact|| over n fresh pairs."""
    e = q = 0.0
    for _ in range(max(1, n // B)):
        a, t = source.batch(B)
        p = sur.forward(a)
        e += float(((p - t) ** 2).sum())
        q += float((t ** 2).sum())
    return math.sqrt(e / q)
