"""Seeded initial magnetisations (SoA layout [3][nz][ny][nx], unit vectors)."""
import numpy as np


def _normalize(m):
    return m / np.sqrt((m * m).sum(axis=0, keepdims=True))


def random_unit(shape, rng):
    """i.i.d. random unit vectors (normal draws, normalised)."""
    return _normalize(rng.standard_normal((3,) + tuple(shape)))


def domain_state(shape, seed, sigma_cells=8.0, tilt=0.1):
    """Perpendicular +/-z domains with small random tilts.

    Gaussian-smoothed noise (std sigma_cells) thresholded at zero chooses
    +z or -z per cell; each cell is then tilted by 0.1*|N(0,1)| rad towards
    a uniformly random azimuth.
    """
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    noise = rng.standard_normal(shape)
    smooth = gaussian_filter(noise, sigma=(0, sigma_cells, sigma_cells),
                             mode="wrap")
    sgn = np.where(smooth >= 0.0, 1.0, -1.0)
    theta = tilt * np.abs(rng.standard_normal(shape))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=shape)
    m = np.empty((3,) + tuple(shape))
    m[0] = np.sin(theta) * np.cos(phi)
    m[1] = np.sin(theta) * np.sin(phi)
    m[2] = sgn * np.cos(theta)
    return m


def stripe_state(shape, seed, width_cells=20, tilt=0.1):
    """Perpendicular stripe domains along y, alternating +z / -z every
    width_cells columns (the same in every layer), the stripe pattern shifted
    by a seeded offset, each cell tilted by tilt*|N(0,1)| rad towards a
    uniformly random azimuth."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    off = int(rng.integers(0, 2 * width_cells))
    sgn1 = np.where(((np.arange(nx) + off) // width_cells) % 2 == 0, 1.0, -1.0)
    sgn = np.broadcast_to(sgn1[None, None, :], shape)
    theta = tilt * np.abs(rng.standard_normal(shape))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=shape)
    m = np.empty((3,) + tuple(shape))
    m[0] = np.sin(theta) * np.cos(phi)
    m[1] = np.sin(theta) * np.sin(phi)
    m[2] = sgn * np.cos(theta)
    return m


def cube_state(shape, seed, tilt_deg=1.0, noise=0.01):
    """+z tilted by tilt_deg towards (1,1,0)/sqrt2, plus small seeded noise."""
    rng = np.random.default_rng(seed)
    th = np.deg2rad(tilt_deg)
    base = np.array([np.sin(th) / np.sqrt(2), np.sin(th) / np.sqrt(2),
                     np.cos(th)])
    m = base[:, None, None, None] + noise * rng.standard_normal((3,) + tuple(shape))
    return _normalize(m)


def initial_state(cfg):
    """List of per-film magnetisations for a config dict from configs.py."""
    d = cfg["desc"]
    shape = (d.nz, d.ny, d.nx)
    kind = cfg["state"]
    if kind == "random":
        rng = np.random.default_rng(cfg["seed"])
        return [random_unit(shape, rng) for _ in range(d.n_films)]
    if kind == "domains":
        seeds = cfg["seed"]
        return [domain_state(shape, seeds[f]) for f in range(d.n_films)]
    if kind == "cube":
        return [cube_state(shape, cfg["seed"])]
    if kind == "stripes":
        seeds = cfg["seed"]
        return [stripe_state(shape, seeds[f]) for f in range(d.n_films)]
    raise ValueError(kind)
