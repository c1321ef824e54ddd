"""Free-space reference for a Gaussian source in a homogeneous medium.

In a homogeneous medium (c = 1, k = omega) the outgoing fundamental
solution of Delta + k^2 is G(r) = -(i/4) H0^(1)(k r) (the Hankel kernel of
Sec. 2.2), outgoing for the time convention e^{-i omega t} under which the
stretching s = (1 + i sigma/omega)^{-1} damps outgoing waves.  For a
unit-mass radial Gaussian of width s_f, the field outside the source is
exactly G(r) times the source's Fourier transform at |xi| = k, i.e.
exp(-k^2 s_f^2 / 2) (Graf's addition theorem averaged over the radial
profile).  The PML discretization should converge to this field at second
order in h away from the source and the absorbing layers.
"""
import numpy as np
from scipy.special import hankel1


def gaussian_field(n, omega, centre, width_in_h=1.5):
    h = 1.0 / (n + 1)
    s = width_in_h * h
    x = h * np.arange(1, n + 1)
    r = np.hypot(x[None, :] - centre[0], x[:, None] - centre[1])
    with np.errstate(all="ignore"):
        u = -0.25j * np.exp(-(omega * s) ** 2 / 2.0) * hankel1(0, omega * r)
    return u, r
