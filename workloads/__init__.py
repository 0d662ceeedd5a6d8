"""Seeded synthetic workloads shared by the GPU binding and the CPU oracle.

This module only *describes* problems (sizes, material constants, drives,
time steps) and *draws* initial magnetisations from seeded generators.  It
holds none of the method's arithmetic: no field, tensor, spline or
integrator code lives here, so that the oracle and the HIP path stay
independent of each other.
"""
from .desc import Desc, Drive, MU0
from .configs import CONFIGS, get_config, slider_mass_damping
from .states import initial_state

__all__ = ["Desc", "Drive", "MU0", "CONFIGS", "get_config", "initial_state",
           "slider_mass_damping"]
