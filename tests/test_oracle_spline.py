"""Pins for the prefiltered cubic B-spline (Sec. III.A)."""
import numpy as np
import pytest
from oracle.spline import beta3, prefilter, interp_1d, interp_3d, prefilter_3d, reflect


def test_partition_of_unity():
    for u in np.linspace(-3, 3, 37):
        k = np.arange(np.floor(u) - 3, np.floor(u) + 4)
        assert np.sum(beta3(u - k)) == pytest.approx(1.0, abs=1e-15)


def test_beta3_values():
    assert beta3(0.0) == pytest.approx(2 / 3)
    assert beta3(1.0) == pytest.approx(1 / 6)
    assert beta3(2.0) == 0.0
    assert beta3(0.5) == pytest.approx(23 / 48)


def test_thomas_equals_dense_solve():
    rng = np.random.default_rng(0)
    for M in (2, 3, 7, 40):
        f = rng.standard_normal(M)
        A = np.zeros((M, M))
        for k in range(M):
            A[k, k] = 4
            if k > 0:
                A[k, k - 1] = 1
            if k < M - 1:
                A[k, k + 1] = 1
        A[0, 1] = 2
        A[M - 1, M - 2] = 2
        c_ref = np.linalg.solve(A / 6.0, f)
        assert np.allclose(prefilter(f), c_ref, rtol=0, atol=1e-13)


def test_node_reproduction():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((4, 29))
    c = prefilter(f, axis=-1)
    got = interp_1d(c, np.arange(29.0))
    assert np.allclose(got, f, rtol=0, atol=1e-13)


def test_cubic_reproduction_interior():
    M = 60
    x = np.arange(M, dtype=float)
    p = lambda t: 0.3 - 0.7 * t + 0.05 * t ** 2 - 0.001 * t ** 3
    c = prefilter(p(x))
    u = np.linspace(25.0, 35.0, 41) + 0.137
    assert np.allclose(interp_1d(c, u), p(u), rtol=0, atol=1e-9 * np.abs(p(x)).max())


def test_shift_by_one_cell_equals_relabel():
    rng = np.random.default_rng(2)
    f = rng.standard_normal(50)
    c = prefilter(f)
    u = np.arange(10, 40) + 1.0
    assert np.allclose(interp_1d(c, u), f[11:41], atol=1e-13)


def test_tensor_spline_reduces_to_1d():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((5, 6, 30))
    c3 = prefilter_3d(f)
    u = np.arange(4, 26) + 0.37
    for (kz, ky) in ((0, 0), (2, 3), (4, 5)):
        c1 = prefilter(f[kz, ky])
        a = interp_3d(c3, u, np.full(u.shape, float(ky)), np.full(u.shape, float(kz)))
        b = interp_1d(c1, u)
        assert np.allclose(a, b, rtol=0, atol=1e-12)


def test_reflect():
    assert list(reflect(np.arange(-3, 9), 5)) == [3, 2, 1, 0, 1, 2, 3, 4, 3, 2, 1, 0]
