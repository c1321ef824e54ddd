"""Seeded synthetic inputs for the 2D PML Helmholtz sweeping solver.

This package builds the inputs of a solve -- velocity fields, right-hand
sides, receiver sets and named problem configurations -- and nothing else.
It holds none of the method's arithmetic (no PML, no stencil, no
factorization), so both the CPU oracle and the GPU path may use it.

The paper's own media (converging lens, waveguide, random medium) and
sources are shown only as figures in Section 3, so the fields here are
closed-form or seeded stand-ins with the same structure: a smooth Gaussian
lens, a smooth Gaussian random field, and Gaussian point sources discretized
at q = 8 points per wavelength.
"""
from .generators import (  # noqa: F401
    grid_points,
    constant_medium,
    lens_medium,
    linear_medium,
    waveguide_medium,
    wave_packet,
    random_field_medium,
    gaussian_source,
    uniform_source_positions,
    bottom_row_sources,
    top_row_receivers,
)
from .configs import WORKLOADS, Workload, get  # noqa: F401
