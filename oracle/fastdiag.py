"""Separable closed form for constant velocity (fast diagonalization).

For c = c0 constant, multiplying the equation at p_{i,j} (eq. helmd) by
(s1 s2)_{i,j} turns the operator into a Kronecker sum

  (L1 (x) I + I (x) L2 + omega^2/c0^2) u = (s1 s2) f,

with the 1D operator (L v)_i = s(x_i) [ s(x_{i-1/2}) (v_{i-1} - v_i)
+ s(x_{i+1/2}) (v_{i+1} - v_i) ] / h^2 and v_0 = v_{n+1} = 0.  Both axes
use the same stretching s, so L1 = L2 = L.  With L = V diag(lambda) V^{-1}
the solution is u = (V (x) V) [(V^{-1} (x) V^{-1}) g / (lambda_i + lambda_j
+ omega^2/c0^2)]: the textbook fast diagonalization (Lynch, Rice and
Thomas).  It builds the operator from its 1D factors, independently of the
2D assembly, and so pins the 2D assembly and the direct solvers.
"""
import numpy as np

from .pml import DEFAULT_C, grid, stretch


def operator_1d(n, omega, pml, C=DEFAULT_C):
    h, x, xh = grid(n)
    eta = pml * h
    s = stretch(x, omega, eta, C)
    sh = stretch(xh, omega, eta, C)
    L = np.zeros((n, n), dtype=np.complex128)
    i = np.arange(n)
    L[i, i] = -s * (sh[:-1] + sh[1:]) / h ** 2
    L[i[1:], i[1:] - 1] = s[1:] * sh[1:-1] / h ** 2
    L[i[:-1], i[:-1] + 1] = s[:-1] * sh[1:-1] / h ** 2
    return L, s


def solve_constant(n, omega, pml, c0, f, C=DEFAULT_C):
    L, s = operator_1d(n, omega, pml, C)
    lam, V = np.linalg.eig(L)
    Vinv = np.linalg.inv(V)
    G = (s[:, None] * s[None, :]) * np.asarray(f, dtype=np.complex128).reshape(n, n)
    Gt = Vinv @ G @ Vinv.T
    Ut = Gt / (lam[:, None] + lam[None, :] + omega ** 2 / c0 ** 2)
    return (V @ Ut @ V.T).reshape(-1)
