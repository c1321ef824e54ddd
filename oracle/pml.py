"""PML profile and coordinate stretching (Sec. 2.1, eq. sigma).

sigma(t) = (C/eta) ((t - eta)/eta)^2        on [0, eta]
         = 0                                on [eta, 1 - eta]
         = (C/eta) ((t - 1 + eta)/eta)^2    on [1 - eta, 1]
s(t)     = (1 + i sigma(t)/omega)^{-1}

The layer width eta is pml * h (the paper gives eta in length units, the
workloads give it in grid points).  The paper leaves the constant C as "an
appropriate positive constant"; the default here is C = 20, which makes the
normal-incidence round trip through the continuous layer decay like
exp(-2C/3) ~ 1.6e-6.
"""
import numpy as np

DEFAULT_C = 20.0


def sigma(t, eta, C=DEFAULT_C):
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    if eta <= 0:
        return out
    lo = t < eta
    hi = t > 1.0 - eta
    out[lo] = (C / eta) * ((t[lo] - eta) / eta) ** 2
    out[hi] = (C / eta) * ((t[hi] - 1.0 + eta) / eta) ** 2
    return out


def stretch(t, omega, eta, C=DEFAULT_C):
    """s(t) = 1 / (1 + i sigma(t) / omega), complex128."""
    return 1.0 / (1.0 + 1j * sigma(t, eta, C) / omega)


def grid(n):
    """h, the interior nodes x_1..x_n and the half nodes x_{1/2}..x_{n+1/2}."""
    h = 1.0 / (n + 1)
    nodes = h * np.arange(1, n + 1, dtype=np.float64)
    halves = h * (np.arange(0, n + 1, dtype=np.float64) + 0.5)
    return h, nodes, halves
