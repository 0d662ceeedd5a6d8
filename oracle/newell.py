"""Cell-averaged demagnetising tensor N (Sec. III.A, Eq. 6).

Eq. (6) writes the demagnetising field of the finite-difference mesh as
H_d(r_i) = -sum_j N(r_i - r_j) M(r_j) with N a 3x3 matrix of "geometrical
coefficients".  We take the cell-averaged tensor of Newell, Williams &
Dunlop (J. Geophys. Res. 98, 9551, 1993): N_xx is a 27-point second
difference of the function f below, N_xy the same difference of g, the
other components by permuting axes.  Convention: N(0) of a cube is +1/3 on
the diagonal, so H = -N M opposes M.

Far from the source the 27-term difference cancels catastrophically in
float64; at |r| >= rc_cells * max(dx, dy, dz) the point-dipole limit
N = V/(4 pi r^3) (I - 3 r r^T / r^2) is used instead.  For cubic cells the
first correction to that limit is O((cell/r)^4).

Pins (tests/test_oracle_newell.py): N_xx+N_yy+N_zz = 1 at r=0 for any
cuboid, 1/3 for a cube; the average of N over all cell pairs of an n^3
cube is 1/3; the far field approaches the dipole; an mpmath evaluation of
the same difference bounds the float64 cancellation error.
"""
import numpy as np

_W = {-1: -1.0, 0: 2.0, 1: -1.0}


def f_newell(x, y, z):
    """Newell's f (even in x, y and z)."""
    x, y, z = np.abs(x), np.abs(y), np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    rxz = np.sqrt(x2 + z2)
    rxy = np.sqrt(x2 + y2)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(rxz > 0, 0.5 * y * (z2 - x2) * np.arcsinh(y / rxz), 0.0)
        t2 = np.where(rxy > 0, 0.5 * z * (y2 - x2) * np.arcsinh(z / rxy), 0.0)
        t3 = np.where(x * R > 0, x * y * z * np.arctan(y * z / (x * R)), 0.0)
    return t1 + t2 - t3 + (2.0 * x2 - y2 - z2) * R / 6.0


def g_newell(x, y, z):
    """Newell's g (odd in x and in y, even in z)."""
    sgn = np.sign(x) * np.sign(y)
    x, y, z = np.abs(x), np.abs(y), np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    rxy = np.sqrt(x2 + y2)
    ryz = np.sqrt(y2 + z2)
    rxz = np.sqrt(x2 + z2)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(rxy > 0, x * y * z * np.arcsinh(z / rxy), 0.0)
        t = t + np.where(ryz > 0, y / 6.0 * (3 * z2 - y2) * np.arcsinh(x / ryz), 0.0)
        t = t + np.where(rxz > 0, x / 6.0 * (3 * z2 - x2) * np.arcsinh(y / rxz), 0.0)
        t = t - np.where(z * R > 0, z ** 3 / 6.0 * np.arctan(x * y / (z * R)), 0.0)
        t = t - np.where(y * R > 0, z * y2 / 2.0 * np.arctan(x * z / (y * R)), 0.0)
        t = t - np.where(x * R > 0, z * x2 / 2.0 * np.arctan(y * z / (x * R)), 0.0)
    t = t - x * y * R / 3.0
    return sgn * t


def _second_difference(fun, X, Y, Z, a, b, c):
    """(1/(4 pi a b c)) sum_{e in {-1,0,1}^3} w(e) fun(X+e1 a, Y+e2 b, Z+e3 c)."""
    acc = 0.0
    for e1 in (-1, 0, 1):
        for e2 in (-1, 0, 1):
            for e3 in (-1, 0, 1):
                w = _W[e1] * _W[e2] * _W[e3]
                acc = acc + w * fun(X + e1 * a, Y + e2 * b, Z + e3 * c)
    return acc / (4.0 * np.pi * a * b * c)


def newell_exact(comp, X, Y, Z, dx, dy, dz):
    """One tensor component from the closed forms (no far-field switch)."""
    X, Y, Z = (np.asarray(v, dtype=np.float64) for v in (X, Y, Z))
    if comp == "xx":
        return _second_difference(f_newell, X, Y, Z, dx, dy, dz)
    if comp == "yy":
        return _second_difference(f_newell, Y, X, Z, dy, dx, dz)
    if comp == "zz":
        return _second_difference(f_newell, Z, Y, X, dz, dy, dx)
    if comp == "xy":
        return _second_difference(g_newell, X, Y, Z, dx, dy, dz)
    if comp == "xz":
        return _second_difference(g_newell, X, Z, Y, dx, dz, dy)
    if comp == "yz":
        return _second_difference(g_newell, Y, Z, X, dy, dz, dx)
    raise ValueError(comp)


_AX = {"x": 0, "y": 1, "z": 2}


def dipole(comp, X, Y, Z, dx, dy, dz):
    """Point-dipole limit V/(4 pi r^3) (delta_ab - 3 r_a r_b / r^2)."""
    r = [np.asarray(v, dtype=np.float64) for v in (X, Y, Z)]
    r2 = r[0] ** 2 + r[1] ** 2 + r[2] ** 2
    a, b = _AX[comp[0]], _AX[comp[1]]
    with np.errstate(divide="ignore", invalid="ignore"):
        val = (dx * dy * dz) / (4.0 * np.pi * r2 ** 1.5) * (
            (1.0 if a == b else 0.0) - 3.0 * r[a] * r[b] / r2)
    return np.where(r2 > 0, val, 0.0)


COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")


_PARITY_AXES = {"xx": (), "yy": (), "zz": (), "xy": (0, 1), "xz": (0, 2),
                "yz": (1, 2)}


def demag_tensor(comp, X, Y, Z, dx, dy, dz, rc_cells=30.0):
    """N_comp at displacements (X, Y, Z) [m]: Newell inside rc, dipole outside.

    Each component has a definite parity in every coordinate (diagonal terms
    even, N_ab odd in a and b), so it is evaluated at (|X|, |Y|, |Z|) and
    multiplied by the parity sign.  This is an identity of the tensor; it
    makes the float64 values exactly symmetric, which the near-field
    cancellation would otherwise break at the 1e-7 level.
    """
    X, Y, Z = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64)
                                    for v in (X, Y, Z)))
    sign = np.ones(X.shape)
    for ax in _PARITY_AXES[comp]:
        sign = sign * np.sign((X, Y, Z)[ax])
    X, Y, Z = np.abs(X), np.abs(Y), np.abs(Z)
    rmax = rc_cells * max(dx, dy, dz)
    far = (X * X + Y * Y + Z * Z) >= rmax * rmax
    out = np.zeros(X.shape)
    near = ~far
    if near.any():
        out[near] = newell_exact(comp, X[near], Y[near], Z[near], dx, dy, dz)
    if far.any():
        out[far] = dipole(comp, X[far], Y[far], Z[far], dx, dy, dz)
    return sign * out


def tensor_matrix(X, Y, Z, dx, dy, dz, rc_cells=30.0):
    """Full symmetric 3x3 tensor, shape (3, 3) + broadcast shape."""
    c = {k: demag_tensor(k, X, Y, Z, dx, dy, dz, rc_cells) for k in COMPONENTS}
    return np.array([[c["xx"], c["xy"], c["xz"]],
                     [c["xy"], c["yy"], c["yz"]],
                     [c["xz"], c["yz"], c["zz"]]])
