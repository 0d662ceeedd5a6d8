"""Local terms of the effective field (Sec. II, text after Eq. 1).

The paper lists exchange, anisotropy, external (Zeeman) and demagnetising
fields and notes that exchange and anisotropy are local (nearest
neighbours / single cell), so they are never interpolated (Sec. II.A).

* exchange   H_ex,i = (2 A / (mu0 Ms)) sum_{nn j} (m_j - m_i) / d^2,
             six nearest neighbours on the cuboid lattice, a neighbour
             outside the magnet is omitted (free boundaries); the two films
             are never exchange coupled;
* anisotropy first-order uniaxial, H_an = (2 Ku / (mu0 Ms)) (m.u) u;
* Zeeman     uniform H_ext.

Pins (tests/test_oracle_fields.py): a helix m = (cos kx, sin kx, 0) has the
exact interior eigenvalue (2 cos(k d) - 2)/d^2; uniform m gives zero
exchange; anisotropy closed form.
"""
import numpy as np
from .constants import MU0


def exchange(desc, m):
    pref = 2.0 * desc.Aex / (MU0 * desc.Ms)
    H = np.zeros_like(m, dtype=np.float64)
    for axis, d in ((3, desc.dx), (2, desc.dy), (1, desc.dz)):
        n = m.shape[axis]
        if n < 2:
            continue
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        diff = (m[tuple(hi)] - m[tuple(lo)]) / (d * d)
        H[tuple(lo)] += diff
        H[tuple(hi)] -= diff
    return pref * H


def anisotropy(desc, m):
    u = np.asarray(desc.u, dtype=np.float64)
    u = u / np.linalg.norm(u) if np.linalg.norm(u) > 0 else u
    pref = 2.0 * desc.Ku / (MU0 * desc.Ms)
    mu = np.einsum("a...,a->...", m, u)
    return pref * mu[None] * u[:, None, None, None]


def zeeman(desc, m):
    h = np.asarray(desc.Hext, dtype=np.float64)
    return np.broadcast_to(h[:, None, None, None], m.shape).copy()
