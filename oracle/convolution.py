"""Lattice sums of Eq. (6) and Eq. (7) on target boxes.

A source film occupies cells [0,nx) x [0,ny) x [0,nz) of its own lattice.
For a target box of lattice points  x in [x0, x0+nwx), y in [y0, y0+nwy),
z in [z0, z0+nwz)  (same lattice spacing, origin of the source film) the
exact linear sum  out(p) = sum_j K(p - r_j) s(r_j)  needs the kernel on the
displacement grid  [x0-(nx-1), x0+nwx-1] x ... .  Two routes compute it:

* `direct_sum`   the O(N^2) double loop, for small pins;
* `WindowSum`    the same sum by FFT: a circular convolution of length equal
                 to the displacement-grid size leaves the "valid" outputs
                 free of wrap-around, so it equals the linear sum exactly
                 up to rounding (Sec. III.A: convolution by FFT).
"""
import numpy as np
from .newell import demag_tensor
from .potential_kernel import potential_kernel


def displacement_axes(desc, box):
    x0, nwx, y0, nwy, z0, nwz = box
    ix = np.arange(x0 - (desc.nx - 1), x0 + nwx)
    iy = np.arange(y0 - (desc.ny - 1), y0 + nwy)
    iz = np.arange(z0 - (desc.nz - 1), z0 + nwz)
    return ix, iy, iz


def displacement_grid(desc, box):
    ix, iy, iz = displacement_axes(desc, box)
    Z, Y, X = np.meshgrid(iz * desc.dz, iy * desc.dy, ix * desc.dx,
                          indexing="ij")
    return X, Y, Z


class WindowSum:
    """out_a(p) = sum_b sum_j K_ab(p - r_j) s_b(j) on a target box, by FFT.

    `kernels` maps (a, b) -> kernel array on the displacement grid
    (shape (Dz, Dy, Dx)); a indexes output channels, b source channels.
    """

    def __init__(self, kernels, src_shape, n_out):
        self.src_shape = tuple(src_shape)
        self.grid_shape = next(iter(kernels.values())).shape
        self.n_out = n_out
        self.khat = {ab: np.fft.rfftn(k, s=self.grid_shape, axes=(0, 1, 2))
                     for ab, k in kernels.items()}

    def __call__(self, src):
        nz, ny, nx = self.src_shape
        shat = {}
        out = []
        for a in range(self.n_out):
            acc = None
            for (aa, b), kh in self.khat.items():
                if aa != a:
                    continue
                if b not in shat:
                    shat[b] = np.fft.rfftn(src[b], s=self.grid_shape, axes=(0, 1, 2))
                term = kh * shat[b]
                acc = term if acc is None else acc + term
            full = np.fft.irfftn(acc, s=self.grid_shape, axes=(0, 1, 2))
            out.append(full[nz - 1:, ny - 1:, nx - 1:])
        return np.array(out)


def direct_sum(kernel_fn, desc, src, box):
    """Brute-force O(N^2) sum.  kernel_fn(X, Y, Z) -> array (n_out, n_src, ...)."""
    x0, nwx, y0, nwy, z0, nwz = box
    nz, ny, nx = src.shape[1:]
    pz, py, px = np.meshgrid(np.arange(z0, z0 + nwz), np.arange(y0, y0 + nwy),
                             np.arange(x0, x0 + nwx), indexing="ij")
    out = None
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                K = kernel_fn((px - i) * desc.dx, (py - j) * desc.dy,
                              (pz - k) * desc.dz)
                term = np.einsum("ab...,b->a...", K, src[:, k, j, i])
                out = term if out is None else out + term
    return out


_PAIRS = {(0, 0): "xx", (0, 1): "xy", (0, 2): "xz", (1, 0): "xy",
          (1, 1): "yy", (1, 2): "yz", (2, 0): "xz", (2, 1): "yz", (2, 2): "zz"}


def demag_window(desc, box, skip_zero=True):
    """WindowSum for H = -Ms sum_j N(p - r_j) m_j on `box` (m = unit vectors)."""
    X, Y, Z = displacement_grid(desc, box)
    comps = {}
    for c in ("xx", "yy", "zz", "xy", "xz", "yz"):
        comps[c] = -desc.Ms * demag_tensor(c, X, Y, Z, desc.dx, desc.dy,
                                           desc.dz, desc.rc_cells)
    kernels = {ab: comps[c] for ab, c in _PAIRS.items()
               if not (skip_zero and not np.any(comps[c]))}
    return WindowSum(kernels, (desc.nz, desc.ny, desc.nx), 3)


def potential_window(desc, box):
    """WindowSum for phi = Ms sum_j S(p - r_j) . m_j on `box` (1 channel)."""
    X, Y, Z = displacement_grid(desc, box)
    S = potential_kernel(X, Y, Z, desc.dx, desc.dy, desc.dz)
    kernels = {(0, b): desc.Ms * S[b] for b in range(3)}
    return WindowSum(kernels, (desc.nz, desc.ny, desc.nx), 1)


def demag_kernel_fn(desc):
    from .newell import tensor_matrix
    return lambda X, Y, Z: -desc.Ms * tensor_matrix(
        X, Y, Z, desc.dx, desc.dy, desc.dz, desc.rc_cells)


def potential_kernel_fn(desc):
    return lambda X, Y, Z: desc.Ms * potential_kernel(
        X, Y, Z, desc.dx, desc.dy, desc.dz)[None]
