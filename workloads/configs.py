"""Named problem configurations.

Each workload fixes the grid (n interior points per side), the angular
frequency omega (q = 8 points per wavelength, as in the paper's 2D tests),
the absorbing-layer width in grid points, a seeded medium, the source
centres, and the compression settings of the layer Schur complements.
"""
from dataclasses import dataclass, field
from typing import Callable, Optional, Tuple

import numpy as np

from . import generators as g


@dataclass
class Workload:
    name: str
    n: int
    omega: float
    pml: int
    medium: Callable[[], np.ndarray]
    source_centres: np.ndarray
    leaf: int
    rank: int
    rank_tol: float
    precision: str                 # "c128" or "c64"
    gmres_tol: float = 1e-6
    dense: bool = False
    receivers: Optional[np.ndarray] = None
    description: str = ""
    extra: dict = field(default_factory=dict)

    def velocity(self):
        return self.medium()

    def sources(self):
        """Right-hand sides, complex128 array (nsrc, n*n)."""
        fs = [g.gaussian_source(self.n, c).reshape(-1) for c in self.source_centres]
        return np.stack(fs, axis=0)


def _centre():
    return np.array([[0.5, 0.5]])


def _helm63():
    n = 63
    return Workload(
        name="helm63_dense_c1", n=n, omega=2 * np.pi * 8, pml=12,
        medium=lambda: g.constant_medium(n), source_centres=_centre(),
        leaf=64, rank=0, rank_tol=0.0, precision="c128", dense=True,
        description="n=63, omega=2pi*8, c=1, PML 12, centre source, dense Schur, c128")


def _helm255(precision="c64"):
    n = 255
    return Workload(
        name="helm255_grf", n=n, omega=2 * np.pi * 32, pml=16,
        medium=lambda: g.random_field_medium(n, seed=1, amplitude=0.3),
        source_centres=_centre(), leaf=16, rank=8, rank_tol=1e-6,
        precision=precision,
        description="n=255, omega=2pi*32, c=1+0.3 GRF(l=0.1, seed 1), PML 16, "
                    "HODLR leaf 16 rank<=8 tol 1e-6, centre source")


def _helm1023():
    n = 1023
    return Workload(
        name="helm1023_lens", n=n, omega=2 * np.pi * 128, pml=24,
        medium=lambda: g.lens_medium(n), source_centres=_centre(),
        leaf=32, rank=8, rank_tol=1e-6, precision="c64",
        description="n=1023, omega=2pi*128, lens c=1-0.4exp(-|x-c|^2/0.1^2), PML 24, "
                    "HODLR leaf 32 rank<=8, c64 factors")


def _helm511_64src():
    n = 511
    return Workload(
        name="helm511_grf_64src", n=n, omega=2 * np.pi * 64, pml=16,
        medium=lambda: g.random_field_medium(n, seed=3, amplitude=0.3),
        source_centres=g.uniform_source_positions(n, 16, 64, seed=4),
        leaf=32, rank=8, rank_tol=1e-6, precision="c64",
        description="n=511, omega=2pi*64, GRF seed 3, 64 sources (seed 4), c64")


def _grad511():
    n = 511
    pml = 16
    return Workload(
        name="grad511", n=n, omega=2 * np.pi * 64, pml=pml,
        medium=lambda: g.constant_medium(n),
        source_centres=g.bottom_row_sources(n, pml, 32),
        receivers=g.top_row_receivers(n, pml, 256),
        leaf=32, rank=8, rank_tol=1e-6, precision="c64",
        description="n=511, omega=2pi*64, c0=1, 32 bottom sources, 256 top receivers; "
                    "data from c_true = 1 + 0.3 GRF(seed 5)",
        extra={"c_true": lambda: g.random_field_medium(n, seed=5, amplitude=0.3),
               "direction_seed": 6})


def mixed_batch():
    """24 instances: 8 each of n = 127, 255, 511, omega = 2 pi (n+1)/8,
    PML 16, media 1 + 0.3 GRF with seeds 100..123, centre sources."""
    out = []
    k = 0
    for n in (127, 255, 511):
        for _ in range(8):
            seed = 100 + k
            out.append(Workload(
                name=f"mixed_{k}_n{n}", n=n, omega=2 * np.pi * (n + 1) / 8, pml=16,
                medium=(lambda n=n, seed=seed: g.random_field_medium(n, seed=seed, amplitude=0.3)),
                source_centres=_centre(), leaf=16 if n <= 255 else 32, rank=8,
                rank_tol=1e-6, precision="c64"))
            k += 1
    return out


WORKLOADS = {
    "helm63_dense_c1": _helm63,
    "helm255_grf": _helm255,
    "helm1023_lens": _helm1023,
    "helm511_grf_64src": _helm511_64src,
    "grad511": _grad511,
}


def get(name, **kw) -> Workload:
    return WORKLOADS[name](**kw)
