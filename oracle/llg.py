"""Landau-Lifshitz-Gilbert right-hand side (Sec. II, Eq. 1).

Eq. (1) is the implicit Gilbert form.  Solved for dm/dt it gives the
Landau-Lifshitz form

   dm/dt = -gamma / (1 + alpha^2) [ m x H + alpha m x (m x H) ].

The sign of the precession term is taken so that damping lowers the
energy: with it, dE/dt = -P_diss of Eq. (4) (pinned in
tests/test_oracle_dynamics.py together with the macrospin closed form
tan(theta/2) = tan(theta0/2) exp(-alpha gamma H t / (1+alpha^2)),
phi = phi0 + gamma H t / (1+alpha^2)).
"""
import numpy as np
from .constants import GAMMA0


def llg_rhs(m, H, alpha, gamma=GAMMA0):
    mxh = np.cross(m, H, axis=0)
    return -gamma / (1.0 + alpha * alpha) * (mxh + alpha * np.cross(m, mxh, axis=0))
