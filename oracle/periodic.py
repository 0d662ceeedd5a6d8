"""Periodic in-plane boundary conditions (Sec. III; Sec. III.A end; Sec. IV.B).

TEST INFRASTRUCTURE ONLY (part of the float64 oracle).

The paper's friction films are periodic in plane: the demagnetising kernel
covers the periodic repetitions of the magnets, and the field data that the
spline needs beyond the domain are copies from the other side instead of a
zero-padded extension.  The paper does not say how the repetitions are
summed; this module takes (reading in the design notes):

* along a periodic axis of n cells the displacement d between two cells is
  reduced to its minimum image w(d) in (-n/2, n/2] (for even n the
  displacement n/2 is the average of the sums at +n/2 and -n/2), and the
  kernel is summed over `pbc_images` repetitions on each side:
      K_per(d) = sum_{|q| <= P} K(w(d) + q n)          (per periodic axis);
* the field of a source on target points along a periodic axis is then the
  circular convolution over one period, and target points outside the
  period take the value of their image (the copy of Sec. III.A);
* along an open axis the zero-padded linear convolution is kept;
* the eddy-current sums (Eq. 9 and the field of the currents) over a
  periodic film take the same image sum of the scalar-potential kernel S of
  Eq. 8 (FilmSWindow), and so does the scalar potential of the potential
  mode (FilmPotWindow): its window rows and columns past the period are
  the values from the other side, the copy the paper describes for the
  potential's extension past the domain.

Pins (tests/test_oracle_periodic.py): the FFT route equals a brute-force loop
over cell pairs and images; a uniform magnetisation gives a field that is the
same in every cell (translation invariance, exact); a uniform perpendicular
film periodic in both axes tends to the infinite-film field H_z = -Ms as the
images grow; shifting the slider by one period leaves its fields unchanged.
The S x v window equals brute-force loops over cells, components and
images, and a uniform dB/dt along z in a film periodic in x and y has no
solenoidal field (tests/test_oracle_periodic_eddy.py).
"""
import numpy as np
from .newell import demag_tensor
from .potential_kernel import potential_kernel

COMPS = ("xx", "yy", "zz", "xy", "xz", "yz")
_PAIRS = {(0, 0): "xx", (0, 1): "xy", (0, 2): "xz", (1, 0): "xy",
          (1, 1): "yy", (1, 2): "yz", (2, 0): "xz", (2, 1): "yz", (2, 2): "zz"}


def min_image(d, n):
    """Minimum image of integer displacements d along a period n, in
    (-n/2, n/2]; returns (w, at_nyquist)."""
    w = np.mod(d, n)
    w = np.where(w > n // 2, w - n, w)
    nyq = (n % 2 == 0) & (w == n // 2)
    return w, nyq


def periodic_kernel(desc, comp, ix, iy, dz_cells):
    """K_per for one tensor component at integer displacements (ix, iy) in
    cells and layer offset dz_cells (broadcast arrays); axes flagged in
    desc.pbc are periodic with desc.pbc_images images on each side."""
    return periodic_sum(desc, lambda X, Y, Z: demag_tensor(comp, X, Y, Z, desc.dx, desc.dy, desc.dz,
                                                           desc.rc_cells), ix, iy, dz_cells)


def periodic_s(desc, comp, ix, iy, dz_cells):
    """The same image sum of the scalar-potential kernel's component comp
    (0, 1, 2 = S_x, S_y, S_z of Eq. 8), the kernel of the eddy-current sums."""
    return periodic_sum(desc, lambda X, Y, Z: potential_kernel(X, Y, Z, desc.dx, desc.dy, desc.dz)[comp],
                        ix, iy, dz_cells)


def periodic_sum(desc, kernel, ix, iy, dz_cells):
    """sum over the images of kernel(X, Y, Z) [displacements in m] at the
    minimum images of the integer displacements (ix, iy) (module docstring)."""
    P = int(desc.pbc_images)
    px = bool(desc.pbc & 1)
    py = bool(desc.pbc & 2)
    ix = np.asarray(ix)
    iy = np.asarray(iy)
    cases_x = [(ix, 1.0)]
    cases_y = [(iy, 1.0)]
    if px:
        w, nyq = min_image(ix, desc.nx)
        # Nyquist: average of +n/2 and -n/2
        cases_x = [(w, np.where(nyq, 0.5, 1.0)), (np.where(nyq, -w, w), np.where(nyq, 0.5, 0.0))]
    if py:
        w, nyq = min_image(iy, desc.ny)
        cases_y = [(w, np.where(nyq, 0.5, 1.0)), (np.where(nyq, -w, w), np.where(nyq, 0.5, 0.0))]
    qx = np.arange(-P, P + 1) if px else np.zeros(1, dtype=int)
    qy = np.arange(-P, P + 1) if py else np.zeros(1, dtype=int)
    out = 0.0
    for wx, cx in cases_x:
        for wy, cy in cases_y:
            wgt = cx * cy
            if not np.any(wgt):
                continue
            # images on two trailing axes, summed afterwards
            X = (np.asarray(wx)[..., None, None] + qx[:, None] * desc.nx) * desc.dx
            Y = (np.asarray(wy)[..., None, None] + qy[None, :] * desc.ny) * desc.dy
            X, Y = np.broadcast_arrays(X, Y)
            Z = np.full(X.shape, dz_cells * desc.dz)
            acc = kernel(X, Y, Z).sum(axis=(-2, -1))
            out = out + wgt * acc
    return out


class FilmWindow:
    """H = -Ms sum_j K_per(p - r_j) m_j of a one-layer film source on target
    points p = (x, y, dz) with x in [x0, x0+nwx), y in [y0, y0+nwy) (source
    lattice indices, any integers) and one layer offset dz (cells).

    Periodic axes: circular convolution over one period by FFT, then the
    target indices taken modulo the period.  Open axes: linear convolution
    on the displacement grid by FFT (as oracle.convolution.WindowSum)."""

    nout = 3  # output channels

    def __init__(self, desc, x0, nwx, y0, nwy, dz_cells):
        self.desc = desc
        self.px, self.py = bool(desc.pbc & 1), bool(desc.pbc & 2)
        nx, ny = desc.nx, desc.ny
        self.box = (x0, nwx, y0, nwy)
        # displacement grids
        if self.px:
            self.gx = np.arange(nx)                       # circular, one period
        else:
            self.gx = np.arange(x0 - (nx - 1), x0 + nwx)
        if self.py:
            self.gy = np.arange(ny)
        else:
            self.gy = np.arange(y0 - (ny - 1), y0 + nwy)
        IY, IX = np.meshgrid(self.gy, self.gx, indexing="ij")
        self.khat = {}
        for (a, b), k in self.kernels(IX, IY, dz_cells).items():
            if np.any(k):
                self.khat[(a, b)] = np.fft.fft2(k)

    def kernels(self, IX, IY, dz_cells):
        """The kernel from source component b to output component a, keyed
        (a, b), on the displacement grid: -Ms N_ab."""
        desc = self.desc
        comp = {c: -desc.Ms * periodic_kernel(desc, c, IX, IY, dz_cells) for c in COMPS}
        return {(a, b): comp[_PAIRS[(a, b)]] for a in range(3) for b in range(3)}

    def __call__(self, m):
        desc = self.desc
        nx, ny = desc.nx, desc.ny
        x0, nwx, y0, nwy = self.box
        Ly, Lx = len(self.gy), len(self.gx)
        shat = [np.fft.fft2(m[b, 0], s=(Ly, Lx)) for b in range(3)]
        out = np.zeros((self.nout, 1, nwy, nwx))
        xs = np.arange(x0, x0 + nwx)
        ys = np.arange(y0, y0 + nwy)
        # index of each target point in the convolution output
        ox = np.mod(xs, nx) if self.px else xs - x0 + (nx - 1)
        oy = np.mod(ys, ny) if self.py else ys - y0 + (ny - 1)
        for a in range(self.nout):
            acc = 0.0
            for b in range(3):
                if (a, b) in self.khat:
                    acc = acc + self.khat[(a, b)] * shat[b]
            if isinstance(acc, float):
                continue
            full = np.real(np.fft.ifft2(acc))
            out[a, 0] = full[np.ix_(oy, ox)]
        return out


# Levi-Civita symbol: (a, b, c) -> eps_abc
EPS = {(0, 1, 2): 1.0, (1, 2, 0): 1.0, (2, 0, 1): 1.0,
       (0, 2, 1): -1.0, (2, 1, 0): -1.0, (1, 0, 2): -1.0}


class FilmSWindow(FilmWindow):
    """out_a = sign * sum_j (S_per(p - r_j) x v_j)_a of a one-layer source
    on the same targets as FilmWindow: the eddy-current sums (Eq. 9 with
    sign +1 for E_sol = S x dB/dt, and the Biot-Savart field of the
    currents with sign -1) over a film periodic in plane."""

    def __init__(self, desc, x0, nwx, y0, nwy, dz_cells, sign):
        self.sign = sign
        super().__init__(desc, x0, nwx, y0, nwy, dz_cells)

    def kernels(self, IX, IY, dz_cells):
        S = [periodic_s(self.desc, b, IX, IY, dz_cells) for b in range(3)]
        ker = {}
        for (a, b, c), e in EPS.items():
            ker[(a, c)] = ker.get((a, c), 0.0) + self.sign * e * S[b]
        return ker


class FilmPotWindow(FilmWindow):
    """The scalar potential phi = Ms sum_j S_per(p - r_j) . m_j of a
    one-layer source (Eqs. 7-8) on the same targets, one output channel:
    the potential of the periodic films, whose values past the period are
    those of the other side (the copy of Sec. III.A end)."""

    nout = 1

    def kernels(self, IX, IY, dz_cells):
        return {(0, b): self.desc.Ms * periodic_s(self.desc, b, IX, IY, dz_cells) for b in range(3)}


def brute_force_pot(desc, m, x0, nwx, y0, nwy, dz_cells):
    """FilmPotWindow by loops over target points and source cells, the
    kernel of each displacement taken from periodic_s."""
    nx, ny = desc.nx, desc.ny
    out = np.zeros((1, 1, nwy, nwx))
    for ty in range(nwy):
        for tx in range(nwx):
            for j in range(ny):
                for i in range(nx):
                    S = np.array([float(periodic_s(desc, b, x0 + tx - i, y0 + ty - j, dz_cells))
                                  for b in range(3)])
                    out[0, 0, ty, tx] += desc.Ms * S @ m[:, 0, j, i]
    return out


def brute_force_s(desc, v, x0, nwx, y0, nwy, dz_cells, sign):
    """FilmSWindow by loops over target points, source cells and the three
    components of the cross product, the kernel of each displacement taken
    from periodic_s."""
    nx, ny = desc.nx, desc.ny
    out = np.zeros((3, 1, nwy, nwx))
    for ty in range(nwy):
        for tx in range(nwx):
            for j in range(ny):
                for i in range(nx):
                    S = np.array([float(periodic_s(desc, b, x0 + tx - i, y0 + ty - j, dz_cells))
                                  for b in range(3)])
                    out[:, 0, ty, tx] += sign * np.cross(S, v[:, 0, j, i])
    return out


def brute_force(desc, m, x0, nwx, y0, nwy, dz_cells):
    """The same sum by loops over target points and source cells, the
    kernel of each displacement (x - i, y - j) taken from periodic_kernel."""
    nx, ny = desc.nx, desc.ny
    dxs = np.arange(x0 - (nx - 1), x0 + nwx)
    dys = np.arange(y0 - (ny - 1), y0 + nwy)
    DY, DX = np.meshgrid(dys, dxs, indexing="ij")
    table = {c: -desc.Ms * periodic_kernel(desc, c, DX, DY, dz_cells) for c in COMPS}
    out = np.zeros((3, 1, nwy, nwx))
    for ty in range(nwy):
        for tx in range(nwx):
            x, y = x0 + tx, y0 + ty
            for j in range(ny):
                for i in range(nx):
                    r, c_ = y - j - dys[0], x - i - dxs[0]
                    for a in range(3):
                        out[a, 0, ty, tx] += sum(table[_PAIRS[(a, b)]][r, c_] * m[b, 0, j, i] for b in range(3))
    return out


class BoxWindow:
    """FilmWindow (or, with potential=True, FilmPotWindow) over a box of
    layers: same call signature and output layout (channels, nwz, nwy, nwx)
    as oracle.convolution.WindowSum on that box."""

    def __init__(self, desc, box, potential=False):
        x0, nwx, y0, nwy, z0, nwz = box
        cls = FilmPotWindow if potential else FilmWindow
        self.layers = [cls(desc, x0, nwx, y0, nwy, z0 + k) for k in range(nwz)]

    def __call__(self, m):
        return np.concatenate([w(m) for w in self.layers], axis=1)


def exchange_periodic(desc, m):
    """Six-neighbour exchange field with periodic neighbours along the
    periodic in-plane axes (free boundaries elsewhere)."""
    from .constants import MU0
    pref = 2.0 * desc.Aex / (MU0 * desc.Ms)
    H = np.zeros_like(m, dtype=np.float64)
    for axis, d, per in ((3, desc.dx, desc.pbc & 1), (2, desc.dy, desc.pbc & 2), (1, desc.dz, 0)):
        n = m.shape[axis]
        if per and n >= 2:
            H += (np.roll(m, 1, axis=axis) + np.roll(m, -1, axis=axis) - 2.0 * m) / (d * d)
            continue
        if n < 2:
            continue
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        diff = (m[tuple(hi)] - m[tuple(lo)]) / (d * d)
        H[tuple(lo)] += diff
        H[tuple(hi)] -= diff
    return pref * H
