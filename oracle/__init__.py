"""FP64 CPU oracle for the moving-magnet micromagnetic hot path.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that
the HIP path is checked against.  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never
does, and it imports nothing from the product package.

Everything is computed in float64 with NumPy/SciPy, following the paper
(Rissanen & Laurson, "Moving magnets in a micromagnetic finite difference
framework") step by step:

  newell.py            demagnetising tensor N of Eq. (6) (Newell et al. 1993)
  potential_kernel.py  scalar-potential kernel S of Eq. (8)
  convolution.py       Eq. (6)/(7) sums on lattice windows (direct and FFT)
  spline.py            prefiltered cubic B-spline interpolation (Sec. III.A)
  fields.py            exchange, anisotropy, Zeeman terms of H_eff (Sec. II)
  llg.py               LLG right-hand side, Eq. (1)
  eddy.py              eddy-current field, Eqs. (9)-(12) (Sec. III.B)
  sim.py               two-film system: cross fields, force Eq. (3),
                       RK4 with the slider equation of motion Eq. (15),
                       diagnostics incl. P_diss Eq. (4)
  dormand_prince.py    adaptive Dormand-Prince RK5(4) of the same system
                       (the paper's RK45 solver, Sec. III)
  periodic.py          periodic in-plane boundaries: image-summed kernels,
                       periodic windows (halo copies), periodic exchange
  divcurl.py           divergence / curl of the interpolated field, Eq. (13)
  applied.py           non-uniform applied field sampled in the moving
                       magnet (Sec. II.A)
  slab.py              two films more than one cell thick, with eddy
                       currents in both (Sec. II.A, III.B, IV.C-D)
  fno.py               learned stray-field operator (Fourier neural
                       operator standing in for the cross term), float64
                       torch with autograd gradients

Parity status of each function is stated in its docstring; functions with
no independent pin say "parity unpinned".
"""
from .constants import MU0, GAMMA_E, GAMMA0
from . import newell, potential_kernel, convolution, spline, fields, llg, sim, fno, dormand_prince, periodic, divcurl
from . import applied, slab

__all__ = ["MU0", "GAMMA_E", "GAMMA0", "newell", "potential_kernel",
           "convolution", "spline", "fields", "llg", "sim", "fno", "dormand_prince",
           "periodic", "divcurl", "applied", "slab"]
