"""PML profile and coordinate stretching (Sec. 2.1, eq. sigma).

sigma(t) = (C/eta) ((t - eta)/eta)^2        on [0, eta]
         = 0                                on [eta, 1 - eta]
         = (C/eta) ((t - 1 + eta)/eta)^2    on [1 - eta, 1]
s(t)     = (1 + i sigma(t)/omega)^{-1}

The layer width eta is pml * h (the paper gives eta in length units, the
workloads give it in grid points).  Each side may have its own width, zero
for a side with the zero Dirichlet condition instead of a layer (the mixed
conditions of Sec. 2.5).  The paper leaves the constant C as "an
appropriate positive constant"; the default here is C = 20, which makes the
normal-incidence round trip through the continuous layer decay like
exp(-2C/3) ~ 1.6e-6.
"""
import numpy as np

DEFAULT_C = 20.0


def sigma(t, eta, C=DEFAULT_C):
    return sigma_sides(t, eta, eta, C)


def sigma_sides(t, eta_lo, eta_hi, C=DEFAULT_C):
    """The profile of eq. sigma with a layer of width eta_lo at t = 0 and
    eta_hi at t = 1; a width of 0 leaves that side without a layer (the
    zero Dirichlet condition of Sec. 2.5 there)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    if eta_lo > 0:
        lo = t < eta_lo
        out[lo] = (C / eta_lo) * ((t[lo] - eta_lo) / eta_lo) ** 2
    if eta_hi > 0:
        hi = t > 1.0 - eta_hi
        out[hi] = (C / eta_hi) * ((t[hi] - 1.0 + eta_hi) / eta_hi) ** 2
    return out


def stretch(t, omega, eta, C=DEFAULT_C):
    """s(t) = 1 / (1 + i sigma(t) / omega), complex128."""
    return stretch_sides(t, omega, eta, eta, C)


def stretch_sides(t, omega, eta_lo, eta_hi, C=DEFAULT_C):
    return 1.0 / (1.0 + 1j * sigma_sides(t, eta_lo, eta_hi, C) / omega)


def grid(n):
    """h, the interior nodes x_1..x_n and the half nodes x_{1/2}..x_{n+1/2}."""
    h = 1.0 / (n + 1)
    nodes = h * np.arange(1, n + 1, dtype=np.float64)
    halves = h * (np.arange(0, n + 1, dtype=np.float64) + 0.5)
    return h, nodes, halves
