"""Scalar-potential kernel S (Sec. III.A, Eq. 8).

S(r_i - r_j) = (1/4pi) integral over cell j of grad' (1/|r - r'|), taken at
the cell centre r_i (the paper evaluates the potential at cell centres,
not corners).  By the divergence theorem the volume integral is a sum over
the six faces of n_f times the integral of 1/|r - r'| over the face, and
each face integral has the closed form

  int int du dv / sqrt(u^2 + v^2 + w^2) = [F(u, v, w)] over the corners,
  F = u asinh(v / sqrt(u^2+w^2)) + v asinh(u / sqrt(v^2+w^2))
      - w atan(u v / (w R)).

The potential of the mesh is phi(r_i) = sum_j S(r_i - r_j) . M_j (Eq. 7) and
H = -grad phi.  Far away S -> V r / (4 pi r^3).  S is evaluated exactly at
every displacement (its face differences lose far fewer digits than the
Newell sums).

Pins (tests/test_oracle_potential.py): adaptive cubature of the defining
integral; S(0) = 0; S odd; far-field limit; -grad of the potential sum
reproduces the Newell field of Eq. (6) far from the source.
"""
import numpy as np


def _F(u, v, w):
    u2, v2, w2 = u * u, v * v, w * w
    R = np.sqrt(u2 + v2 + w2)
    ruw = np.sqrt(u2 + w2)
    rvw = np.sqrt(v2 + w2)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(ruw > 0, u * np.arcsinh(v / ruw), 0.0)
        t = t + np.where(rvw > 0, v * np.arcsinh(u / rvw), 0.0)
        t = t - np.where((w != 0) & (R > 0), w * np.arctan(u * v / (w * R)), 0.0)
    return t


def _rect(u1, u2, v1, v2, w):
    """int_{u1}^{u2} int_{v1}^{v2} du dv / sqrt(u^2+v^2+w^2)."""
    return _F(u2, v2, w) - _F(u1, v2, w) - _F(u2, v1, w) + _F(u1, v1, w)


def _axis_component(A, B, C, a, b, c):
    """Component along the first axis; (A,B,C) displacement, (a,b,c) cell."""
    def face(w):
        return _rect(-b / 2 - B, b / 2 - B, -c / 2 - C, c / 2 - C, w)
    return (face(A - a / 2) - face(A + a / 2)) / (4.0 * np.pi)


def potential_kernel(X, Y, Z, dx, dy, dz):
    """(S_x, S_y, S_z) at displacement (X, Y, Z) [m] (broadcast arrays)."""
    X, Y, Z = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64)
                                    for v in (X, Y, Z)))
    sx = _axis_component(X, Y, Z, dx, dy, dz)
    sy = _axis_component(Y, X, Z, dy, dx, dz)
    sz = _axis_component(Z, X, Y, dz, dx, dy)
    return np.array([sx, sy, sz])
