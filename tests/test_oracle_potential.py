"""Pins for the scalar-potential kernel S (Eq. 8)."""
import numpy as np
import pytest
from scipy import integrate
from oracle.potential_kernel import potential_kernel


def cubature(X, Y, Z, dx, dy, dz, comp):
    def g(z, y, x):
        r = np.array([X - x, Y - y, Z - z])
        return r[comp] / np.sum(r * r) ** 1.5
    v, _ = integrate.tplquad(g, -dx / 2, dx / 2, -dy / 2, dy / 2, -dz / 2, dz / 2,
                             epsabs=1e-13, epsrel=1e-11)
    return v / (4 * np.pi)


@pytest.mark.parametrize("p", [(1.3, 0.2, -0.7), (2.0, 1.0, 0.0), (0.9, 0.0, 1.1),
                               (5.0, -3.0, 2.0), (0.0, 1.0, 2.0)])
def test_against_cubature(p):
    cell = (1.0, 1.3, 0.8)
    S = potential_kernel(*p, *cell)
    for c in range(3):
        assert S[c] == pytest.approx(cubature(*p, *cell, c), rel=1e-9, abs=1e-13)


def test_origin_and_oddness():
    S0 = potential_kernel(0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    assert np.all(np.abs(S0) < 1e-16)
    p = np.array([2.0, -1.0, 3.0])
    assert np.allclose(potential_kernel(*(-p), 1, 1, 1), -potential_kernel(*p, 1, 1, 1),
                       rtol=1e-13, atol=0)


def test_far_field():
    p = np.array([40.0, -25.0, 13.0])
    r = np.linalg.norm(p)
    S = potential_kernel(*p, 1.0, 1.0, 1.0)
    ref = p / (4 * np.pi * r ** 3)
    assert np.allclose(S, ref, rtol=1e-5)


def test_gradient_matches_tensor_far_away():
    """-grad of the potential of one cell ~ the Newell field (both -> dipole)."""
    from oracle.newell import tensor_matrix
    h = 1e-3
    p = np.array([9.0, 4.0, 3.0])
    m = np.array([0.3, -0.5, 0.81])
    grad = np.zeros(3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        grad[a] = (potential_kernel(*(p + e), 1, 1, 1) @ m
                   - potential_kernel(*(p - e), 1, 1, 1) @ m) / (2 * h)
    H_pot = -grad
    H_ten = -tensor_matrix(*p, 1.0, 1.0, 1.0) @ m
    # point-evaluated vs cell-averaged target: agree to O((d/r)^2)
    assert np.allclose(H_pot, H_ten, rtol=0, atol=2e-2 * np.abs(H_ten).max())
