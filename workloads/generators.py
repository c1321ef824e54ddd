"""Seeded generators for media, sources and receivers.

Grid convention (Section 2.1, Discretization): the unit square is sampled
with spacing h = 1/(n+1); the interior points are p_{i,j} = (i h, j h) for
1 <= i, j <= n.  Every 2D field is an (n, n) array indexed [j-1, i-1], so
that its row-major flattening is the paper's unknown ordering (row by row,
x1 index fastest).
"""
import numpy as np
from scipy.ndimage import gaussian_filter


def grid_points(n):
    """Interior coordinates x_1..x_n = h, 2h, ..., n h with h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    return h * np.arange(1, n + 1, dtype=np.float64)


def _mesh(n):
    x = grid_points(n)
    x1 = x[None, :]          # varies along the fast (i) axis
    x2 = x[:, None]          # varies along the slow (j) axis
    return x1, x2


def constant_medium(n, value=1.0):
    """Homogeneous velocity c = value."""
    return np.full((n, n), float(value), dtype=np.float64)


def lens_medium(n, depth=0.4, width=0.1, centre=(0.5, 0.5)):
    """Converging lens c = 1 - depth * exp(-|x - centre|^2 / width^2).

    A smooth Gaussian low-velocity region, the same kind of medium as the
    paper's first test velocity field (Section 3, PML tests).
    """
    x1, x2 = _mesh(n)
    r2 = (x1 - centre[0]) ** 2 + (x2 - centre[1]) ** 2
    return 1.0 - depth * np.exp(-r2 / width ** 2)


def linear_medium(n, base=0.5, slope=1.0):
    """c = base + slope * x2: the velocity of the paper's sweep-direction
    example (Sec. 3, dependence on the sweep direction), 1/2 + x2."""
    x1, x2 = _mesh(n)
    return np.broadcast_to(base + slope * x2, (n, n)).astype(np.float64).copy()


def waveguide_medium(n, depth=0.4, width=0.1, centre=0.5):
    """A vertical waveguide c = 1 - depth * exp(-(x1 - centre)^2 / width^2): a
    low-velocity channel along x2, the kind of medium of the paper's
    depth-extrapolation example (Sec. 3, other boundary conditions)."""
    x1, x2 = _mesh(n)
    return np.broadcast_to(1.0 - depth * np.exp(-((x1 - centre) ** 2) / width ** 2), (n, n)).astype(np.float64).copy()


def wave_packet(n, centre, direction, omega, width=None):
    """Gaussian wave packet f = exp(-|x - x0|^2 / (2 s^2)) exp(i omega d.(x - x0)) / (2 pi s^2)
    with unit direction d and width s of one wavelength 2 pi / omega unless
    given, sampled at the interior points (complex128, (n, n))."""
    s = 2 * np.pi / omega if width is None else width
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    x1, x2 = _mesh(n)
    dx1, dx2 = x1 - centre[0], x2 - centre[1]
    env = np.exp(-(dx1 ** 2 + dx2 ** 2) / (2 * s * s)) / (2 * np.pi * s * s)
    return (env * np.exp(1j * omega * (d[0] * dx1 + d[1] * dx2))).astype(np.complex128)


def random_field_medium(n, seed, amplitude=0.3, corr_length=0.1):
    """Smooth Gaussian random field c = 1 + amplitude * g, max |g| = 1.

    White noise N(0, 1) on the n x n grid from numpy's PCG64 generator
    seeded with `seed`, filtered by a Gaussian kernel of standard deviation
    corr_length / sqrt(2) (so the covariance decays like
    exp(-r^2 / (2 corr_length^2))), reflected at the edges, and normalized
    so that c lies in [1 - amplitude, 1 + amplitude].
    """
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n))
    g = gaussian_filter(noise, sigma=corr_length / (np.sqrt(2.0) * h), mode="reflect")
    g /= np.max(np.abs(g))
    return 1.0 + amplitude * g


def gaussian_source(n, centre, width_in_h=1.5):
    """Unit-mass Gaussian point source sampled at the interior points.

    f(x) = exp(-|x - x0|^2 / (2 s^2)) / (2 pi s^2) with s = width_in_h * h.
    Returned as complex128, shape (n, n), indexed [j-1, i-1].
    """
    h = 1.0 / (n + 1)
    s = width_in_h * h
    x1, x2 = _mesh(n)
    r2 = (x1 - centre[0]) ** 2 + (x2 - centre[1]) ** 2
    f = np.exp(-r2 / (2.0 * s * s)) / (2.0 * np.pi * s * s)
    return f.astype(np.complex128)


def _inner_range(n, pml, margin=6):
    h = 1.0 / (n + 1)
    lo = (pml + margin) * h
    return lo, 1.0 - lo


def uniform_source_positions(n, pml, count, seed, margin=6):
    """`count` source centres drawn uniformly in the square kept `margin`
    grid points clear of the absorbing layer on every side."""
    lo, hi = _inner_range(n, pml, margin)
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(count, 2))


def bottom_row_sources(n, pml, count, margin=6):
    """`count` source centres on the line x2 = (pml + margin) h, evenly
    spaced in x1 over the same clear range."""
    lo, hi = _inner_range(n, pml, margin)
    x1 = np.linspace(lo, hi, count)
    return np.stack([x1, np.full(count, lo)], axis=1)


def top_row_receivers(n, pml, count, margin=6):
    """Flat indices of `count` receivers on grid row j = n + 1 - (pml + margin).

    The columns are the nearest grid columns to `count` evenly spaced x1
    positions over the clear range.  The flat index is (j-1) n + (i-1).
    """
    h = 1.0 / (n + 1)
    lo, hi = _inner_range(n, pml, margin)
    j = n + 1 - (pml + margin)
    cols = np.rint(np.linspace(lo, hi, count) / h).astype(np.int64)
    cols = np.clip(cols, 1, n)
    return (j - 1) * n + (cols - 1)
