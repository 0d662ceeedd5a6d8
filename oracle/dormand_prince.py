"""Adaptive Dormand-Prince RK5(4) for (m_base, m_slider, x_s, v_s) (Sec. III).

TEST INFRASTRUCTURE ONLY (part of the float64 oracle).

The paper integrates the LLG equation together with the slider's Newton
equation (Eq. 15) in MuMax3's adaptive RK45 Dormand-Prince solver (Sec. III,
Sec. IV.D).  It gives no tolerances, error norm or step-size rule, so this
module takes the textbook method:

* the seven-stage Dormand-Prince pair (Dormand & Prince, J. Comput. Appl.
  Math. 6, 19, 1980), advancing with the fifth-order solution (local
  extrapolation) and estimating the error from the embedded fourth-order one;
* every stage evaluates H_eff at its own (m, x_s, v_s, t) and the slider's
  force there, exactly as the classic RK4 of sim.System;
* error norm: the largest of
    max over cells of |e_m| (Euclidean norm of the error vector of m),
    |e_x| / dx              (slider position error in cells),
    |e_v| h / dx            (the displacement the velocity error makes over
                             the step, in cells),
  divided by the tolerance; the step is accepted when this is <= 1;
* step size: h_new = h * min(5, max(0.2, 0.9 err^(-1/5))) (at most h after a
  rejection), the standard controller of Hairer, Norsett & Wanner, Solving
  ODEs I, Sec. II.4, clipped so that the run ends exactly at t_end;
* after an accepted step m is renormalised and s_int re-seated, as after an
  RK4 step; the next step evaluates its first stage afresh (the renormalised
  state is not the one the seventh stage saw, so no first-same-as-last).

Pins (tests/test_oracle_dormand_prince.py): the tableau's order conditions up
to order five and the embedded pair's up to four; fifth-order convergence of
fixed steps on the macrospin closed form; the adaptive run meets the
macrospin closed form within a small multiple of the tolerance; a constant
velocity drive is integrated exactly; the spring drive's critically damped
closed form.
"""
import math
import numpy as np

# Butcher tableau of the Dormand-Prince pair (published rational constants).
C = (0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0)
A = (
    (),
    (1.0 / 5.0,),
    (3.0 / 40.0, 9.0 / 40.0),
    (44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0),
    (19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0),
    (9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0),
    (35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0),
)
B5 = (35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0)
B4 = (5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0, -92097.0 / 339200.0,
      187.0 / 2100.0, 1.0 / 40.0)
E = tuple(b5 - b4 for b5, b4 in zip(B5, B4))

SAFETY, FAC_MIN, FAC_MAX = 0.9, 0.2, 5.0


def new_step(h, err, accepted):
    """Next step size from the error ratio err (<= 1 accepted)."""
    fac = FAC_MAX if err == 0.0 else min(FAC_MAX, max(FAC_MIN, SAFETY * err ** -0.2))
    if not accepted:
        fac = min(fac, 1.0)
    return h * fac


def attempt(system, h):
    """One Dormand-Prince attempt of size h from the system's state.

    Returns (y5 as ([m per film], x, v), error ratio, stage derivatives).
    The system is not modified.
    """
    m0, x0, v0, t0 = system.m, system.x, system.v, system.t
    ks = []
    for i in range(7):
        if i == 0:
            mi, xi, vi = m0, x0, v0
        else:
            mi = [m + h * sum(A[i][j] * ks[j][0][f] for j in range(i))
                  for f, m in enumerate(m0)]
            xi = x0 + h * sum(A[i][j] * ks[j][1] for j in range(i))
            vi = v0 + h * sum(A[i][j] * ks[j][2] for j in range(i))
        ks.append(system.derivative(mi, xi, vi, t0 + C[i] * h))
    y5 = mi, xi, vi      # the seventh stage's state is the fifth-order solution
    em = [h * sum(E[j] * ks[j][0][f] for j in range(7)) for f in range(len(m0))]
    ex = h * sum(E[j] * ks[j][1] for j in range(7))
    ev = h * sum(E[j] * ks[j][2] for j in range(7))
    dx = system.desc.dx
    err_m = max(float(np.sqrt((e * e).sum(axis=0)).max()) for e in em)
    err = max(err_m, abs(ex) / dx, abs(ev) * h / dx)
    return y5, err, ks


def step(system, h, tol):
    """Try one step of size h.  Returns (accepted, next h)."""
    (m5, x5, v5), err, _ = attempt(system, h)
    ratio = err / tol
    ok = ratio <= 1.0
    if ok:
        system.m = [m / np.sqrt((m * m).sum(axis=0, keepdims=True)) for m in m5]
        system.x, system.v = x5, v5
        system.t = system.t + h
        system.s_int = int(math.floor(system.x / system.desc.dx))
        system.step_count += 1
    return ok, new_step(h, ratio, ok)


END_REL = 1e-9   # the run has reached t_end when t_end - t <= END_REL * t_end


def run(system, t_end, h0, tol, max_attempts=100000):
    """Integrate to t_end (the last step clipped to land on it).

    Returns (accepted, rejected, next h)."""
    h = h0
    acc = rej = 0
    while t_end - system.t > END_REL * t_end and acc + rej < max_attempts:
        hh = min(h, t_end - system.t)
        ok, h = step(system, hh, tol)
        if ok:
            acc += 1
            if t_end - system.t <= END_REL * t_end:
                system.t = t_end
        else:
            rej += 1
    return acc, rej, h
