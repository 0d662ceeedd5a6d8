"""Pins for the oracle's adaptive Dormand-Prince RK5(4) (Sec. III: the
paper's RK45 solver with the slider's equation of motion)."""
import math
from fractions import Fraction
import numpy as np
import pytest
from workloads import Desc, Drive
from workloads.states import random_unit, domain_state
from oracle import dormand_prince as dp
from oracle.constants import GAMMA0
from oracle.sim import System, SPRING, VELOCITY


# ------------------------------------------------------------- order conditions
# Rooted trees as sorted tuples of subtrees; the single node is ().  For a
# method (A, b, c) the tree t = [t1..tk] needs sum_i b_i Phi_i(t) = 1/gamma(t),
# Phi_i(t) = prod_m sum_j a_ij Phi_j(t_m), gamma(t) = |t| prod_m gamma(t_m)
# (Butcher; Hairer, Norsett & Wanner I, Sec. II.2).

def trees(order):
    """All rooted trees with `order` nodes."""
    if order == 1:
        return [()]
    out = set()

    def forests(n, smallest):
        # multisets of trees with n nodes in total, in non-decreasing order
        if n == 0:
            yield ()
            return
        for k in range(1, n + 1):
            for t in sorted(trees(k)):
                if (k, t) < smallest:
                    continue
                for rest in forests(n - k, (k, t)):
                    yield (t,) + rest
    for f in forests(order - 1, (0, ())):
        out.add(tuple(sorted(f)))
    return sorted(out)


def size(t):
    return 1 + sum(size(s) for s in t)


def gamma(t):
    g = size(t)
    for s in t:
        g *= gamma(s)
    return g


def phi(t, A, i):
    v = Fraction(1)
    for s in t:
        v *= sum((Fraction(A[i][j]).limit_denominator(10 ** 7) * phi(s, A, j) for j in range(i)), Fraction(0))
    return v


def test_tree_counts():
    assert [len(trees(p)) for p in range(1, 6)] == [1, 1, 2, 4, 9]


def test_row_sums_equal_nodes():
    for i in range(7):
        assert abs(sum(dp.A[i]) - dp.C[i]) < 1e-15


@pytest.mark.parametrize("b,p", [(dp.B5, 5), (dp.B4, 4)])
def test_order_conditions(b, p):
    for q in range(1, p + 1):
        for t in trees(q):
            lhs = sum(Fraction(b[i]).limit_denominator(10 ** 7) * phi(t, dp.A, i) for i in range(7))
            assert lhs == Fraction(1, gamma(t)), (q, t)


def test_fourth_order_pair_is_not_fifth_order():
    # the embedded solution must differ at order five (else no error estimate)
    bad = [t for t in trees(5)
           if sum(Fraction(dp.B4[i]).limit_denominator(10 ** 7) * phi(t, dp.A, i) for i in range(7))
           != Fraction(1, gamma(t))]
    assert bad


def test_pins_reject_a_mistyped_coefficient(monkeypatch):
    A = [list(r) for r in dp.A]
    A[4][2] = 64448.0 / 6562.0
    fails = [t for q in range(1, 6) for t in trees(q)
             if sum(Fraction(dp.B5[i]).limit_denominator(10 ** 7) * phi(t, A, i) for i in range(7))
             != Fraction(1, gamma(t))]
    assert fails


# ------------------------------------------------------------- the integrator
def macrospin(alpha=0.1, H=1e5, th0=0.5, ph0=0.2):
    d = Desc(n_films=1, nx=1, ny=1, nz=1, dx=3e-9, dy=3e-9, dz=3e-9, Ms=8e5,
             Aex=1e-11, alpha=alpha, Hext=(0.0, 0.0, H))
    m = np.zeros((3, 1, 1, 1))
    m[:, 0, 0, 0] = [math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0), math.cos(th0)]
    return System(d, Drive(), [m])


def macrospin_exact(t, alpha=0.1, H=1e5, th0=0.5, ph0=0.2):
    g = GAMMA0 / (1 + alpha ** 2)
    th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * g * H * t))
    ph = ph0 + g * H * t
    return np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])


def test_fixed_steps_converge_at_fifth_order():
    T = 4e-11
    errs = []
    for n in (10, 20):
        s = macrospin()
        for _ in range(n):
            ok, _ = dp.step(s, T / n, float("inf"))
            assert ok
        errs.append(np.abs(s.m[0][:, 0, 0, 0] - macrospin_exact(s.t)).max())
    assert 24 < errs[0] / errs[1] < 40       # 2^5 = 32


def test_adaptive_run_meets_the_tolerance():
    T = 2e-10
    out = []
    for tol in (1e-6, 1e-8):
        s = macrospin()
        acc, rej, h = dp.run(s, T, 1e-14, tol)
        assert s.t == T
        err = np.abs(s.m[0][:, 0, 0, 0] - macrospin_exact(T)).max()
        out.append((tol, acc, rej, err))
        assert err <= 10 * tol
    assert out[1][1] > out[0][1]                 # tighter tolerance, more steps


def test_rejected_step_leaves_the_state():
    s = macrospin()
    m0 = s.m[0].copy()
    ok, h = dp.step(s, 1e-11, 1e-12)
    assert not ok and h < 1e-11
    assert s.t == 0.0 and np.array_equal(s.m[0], m0)


def two_film(mode, **kw):
    d = Desc(n_films=2, nx=12, ny=8, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, gap_cells=1,
             Ms=1.1e6, Aex=1.5e-11, alpha=0.1, Ku=8e5)
    m = [domain_state((1, 8, 12), 3), domain_state((1, 8, 12), 4)]
    return System(d, Drive(mode=mode, **kw), m)


def test_velocity_drive_is_exact_under_adaptive_steps():
    s = two_film(VELOCITY, v_d=4.0, x0=0.9 * 2e-9)
    acc, rej, _ = dp.run(s, 1e-12, 1e-14, 1e-5)
    assert acc > 3
    assert s.x == pytest.approx(0.9 * 2e-9 + 4.0 * 1e-12, rel=1e-13)
    assert s.s_int == 0


class NoCross(System):
    def cross_fields(self, m_b, m_s, x, s_int, want_force=True):
        z = np.zeros_like(m_b)
        return z, z, np.zeros(3)


def test_spring_drive_critical_damping_closed_form():
    d = Desc(n_films=2, nx=4, ny=4, nz=1, dx=2e-9, dy=2e-9, dz=2e-9, Ms=1e6, alpha=0.1)
    k, M = 1e-3, 1e-20
    w0 = math.sqrt(k / M)
    # uniform +z films carry no torque: the slider alone sets the steps
    m = np.zeros((3, 1, 4, 4))
    m[2] = 1.0
    s = NoCross(d, Drive(mode=SPRING, v_d=1.0, k=k, mass=M, gamma_v=2 * w0), [m, m.copy()])
    acc, rej, _ = dp.run(s, 2e-9, 1e-13, 1e-7)
    t = s.t
    x_ref = t - 2 / w0 + (2 / w0 + t) * math.exp(-w0 * t)
    # the slider's error terms are in the norm: its trajectory follows the
    # tolerance (in cells) rather than the magnetisation's step size
    assert abs(s.x - x_ref) / d.dx < 1e-5
    assert s.s_int == math.floor(s.x / d.dx)
