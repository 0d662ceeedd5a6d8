"""Physical constants (SI).

The paper names gamma but gives no value (Sec. II, Eq. 1).  Eq. (1) and
Eq. (4) use gamma acting on a field in A/m, so gamma = mu0 * gamma_e with
the electron gyromagnetic ratio gamma_e = 1.7595e11 rad/(s T).
"""
import math

MU0 = 4e-7 * math.pi
GAMMA_E = 1.7595e11
GAMMA0 = MU0 * GAMMA_E
