"""Prefiltered cubic B-spline interpolation (Sec. III.A).

The paper interpolates the stray field (or its scalar potential) of one
magnet at the sub-cell position of the other with C2 cubic B-splines whose
coefficients come from a prefilter, so that the spline passes through the
lattice data.  Data are taken on a window that extends `halo` cells past
the magnet along the motion axis (the paper uses four).

Definition used here.  Window samples f_0..f_{M-1}; coefficients c solve

   (4 c_0 + 2 c_1) / 6 = f_0
   (c_{k-1} + 4 c_k + c_{k+1}) / 6 = f_k          0 < k < M-1
   (2 c_{M-2} + 4 c_{M-1}) / 6 = f_{M-1}

(whole-sample mirror boundaries), solved with the Thomas algorithm.  The
interpolant is s(u) = sum_k c_k beta3(u - k) with the mirror-extended
coefficients c_{-k} = c_k, c_{M-1+k} = c_{M-1-k}, and

   beta3(t) = 2/3 - t^2 + |t|^3 / 2     |t| <= 1
            = (2 - |t|)^3 / 6           1 <= |t| <= 2
            = 0                         otherwise.

Pins (tests/test_oracle_spline.py): node reproduction s(k) = f_k; partition
of unity; cubic polynomials reproduced away from the window ends; the
tensor-product 64-tap evaluation reduces to the 1-D one when only one
coordinate is fractional; the Thomas solve equals a dense solve.
"""
import numpy as np


def beta3(t):
    a = np.abs(np.asarray(t, dtype=np.float64))
    return np.where(a <= 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                    np.where(a <= 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def prefilter(f, axis=-1):
    """Spline coefficients of the mirror-bounded system along `axis`."""
    f = np.moveaxis(np.asarray(f, dtype=np.float64), axis, -1)
    M = f.shape[-1]
    if M == 1:
        return np.moveaxis(f.copy(), -1, axis)
    sub = np.full(M, 1.0 / 6.0)
    diag = np.full(M, 4.0 / 6.0)
    sup = np.full(M, 1.0 / 6.0)
    sup[0] = 2.0 / 6.0
    sub[M - 1] = 2.0 / 6.0
    # forward elimination
    cp = np.empty(M)
    dp = np.empty(f.shape)
    cp[0] = sup[0] / diag[0]
    dp[..., 0] = f[..., 0] / diag[0]
    for k in range(1, M):
        den = diag[k] - sub[k] * cp[k - 1]
        cp[k] = sup[k] / den if k < M - 1 else 0.0
        dp[..., k] = (f[..., k] - sub[k] * dp[..., k - 1]) / den
    # back substitution
    c = np.empty(f.shape)
    c[..., M - 1] = dp[..., M - 1]
    for k in range(M - 2, -1, -1):
        c[..., k] = dp[..., k] - cp[k] * c[..., k + 1]
    return np.moveaxis(c, -1, axis)


def reflect(k, M):
    """Whole-sample mirror index into [0, M)."""
    k = np.asarray(k)
    if M == 1:
        return np.zeros_like(k)
    P = 2 * M - 2
    k = np.mod(k, P)
    return np.where(k > M - 1, P - k, k)


def interp_1d(c, u, axis=-1):
    """s(u) along `axis` for the positions u (1-D array)."""
    c = np.moveaxis(np.asarray(c, dtype=np.float64), axis, -1)
    M = c.shape[-1]
    u = np.asarray(u, dtype=np.float64)
    k0 = np.floor(u).astype(np.int64)
    out = np.zeros(c.shape[:-1] + u.shape)
    for t in (-1, 0, 1, 2):
        k = k0 + t
        out += c[..., reflect(k, M)] * beta3(u - k)
    return np.moveaxis(out, -1, axis) if u.ndim == 1 else out


def interp_3d(c, u, v, w):
    """64-tap tensor-product spline at points (u, v, w) of c[z, y, x].

    u indexes x (last axis), v indexes y, w indexes z; c holds coefficients
    already prefiltered along all three axes.
    """
    c = np.asarray(c, dtype=np.float64)
    Mz, My, Mx = c.shape
    u, v, w = (np.asarray(a, dtype=np.float64) for a in (u, v, w))
    ku, kv, kw = (np.floor(a).astype(np.int64) for a in (u, v, w))
    out = np.zeros(u.shape)
    for tz in (-1, 0, 1, 2):
        for ty in (-1, 0, 1, 2):
            for tx in (-1, 0, 1, 2):
                wgt = (beta3(w - (kw + tz)) * beta3(v - (kv + ty))
                       * beta3(u - (ku + tx)))
                out += wgt * c[reflect(kw + tz, Mz), reflect(kv + ty, My),
                               reflect(ku + tx, Mx)]
    return out


def prefilter_3d(f):
    return prefilter(prefilter(prefilter(f, axis=2), axis=1), axis=0)


def linear_1d(f, u, axis=-1):
    """Linear interpolation of the samples f (no prefilter) at positions u:
    (1 - t) f[k] + t f[k + 1], k = floor(u), t = u - k, mirror indices
    (the comparison interpolant of Sec. IV.A)."""
    f = np.moveaxis(np.asarray(f, dtype=np.float64), axis, -1)
    M = f.shape[-1]
    u = np.asarray(u, dtype=np.float64)
    k0 = np.floor(u).astype(np.int64)
    t = u - k0
    out = f[..., reflect(k0, M)] * (1.0 - t) + f[..., reflect(k0 + 1, M)] * t
    return np.moveaxis(out, -1, axis) if u.ndim == 1 else out
