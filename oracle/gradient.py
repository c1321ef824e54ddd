"""Receiver misfit and its gradient with respect to the velocity.

J(c) = 1/2 sum_s || P u_s(c) - d_s ||^2, with A(c) u_s = f_s and P the
restriction to receiver points.  The velocity enters A only through the
centre coefficient omega^2/((s1 s2) c^2) of eq. helmd, so
dA/dc_{ij} = -2 omega^2 / ((s1 s2)_{ij} c_{ij}^3) on the diagonal.  With
g_s = P^t (P u_s - d_s) (the derivative of J with respect to the real and
imaginary parts of u_s) and A = A^t (symmetric operator, Sec. 2.1), the
adjoint field is mu_s = A^{-1} conj(g_s) and

  dJ/dc_{ij} = sum_s Re( mu_{s,ij} u_{s,ij} 2 omega^2 / ((s1 s2)_{ij} c_{ij}^3) ),

the real part taken of the whole product because s1 s2 is complex inside
the PML.  Every solve here is a sparse direct solve.
"""
import numpy as np

from . import assemble, direct
from .pml import DEFAULT_C


def forward(c, omega, pml, F, C=DEFAULT_C):
    st = assemble.stencil(c, omega, pml, C)
    lu = direct.SparseLU(st)
    return st, lu, lu.solve(F)


def misfit(c, omega, pml, F, receivers, data, C=DEFAULT_C):
    _, _, U = forward(c, omega, pml, F, C)
    r = U[:, receivers] - data
    return 0.5 * np.sum(np.abs(r) ** 2)


def adjoint_gradient(c, omega, pml, F, receivers, data, C=DEFAULT_C):
    """Returns (J, dJ/dc as an (n, n) array)."""
    J, grad, _, _ = adjoint_state(c, omega, pml, F, receivers, data, C)
    return J, grad


def adjoint_state(c, omega, pml, F, receivers, data, C=DEFAULT_C):
    """Returns (J, dJ/dc, the fields U, the adjoint fields Mu).

    J is linear-quadratic in the sources as well: u_s = A^{-1} f_s gives
    dJ = Re sum_s mu_s^t df_s (A = A^t), so the gradient with respect to the
    real and imaginary parts of f_s, packed as dJ/dRe f + i dJ/dIm f, is
    conj(mu_s)."""
    st, lu, U = forward(c, omega, pml, F, C)
    n = st.n
    r = U[:, receivers] - data
    J = 0.5 * np.sum(np.abs(r) ** 2)
    G = np.zeros_like(U)
    G[:, receivers] = r
    Mu = lu.solve(np.conj(G))
    dD = 2.0 * omega ** 2 / (st.s1s2 * st.c ** 3)
    grad = np.real(Mu.reshape(-1, n, n) * U.reshape(-1, n, n) * dD[None]).sum(axis=0)
    return J, grad, U, Mu


def central_difference(c, omega, pml, F, receivers, data, direction, eps, C=DEFAULT_C):
    """(J(c + eps v) - J(c - eps v)) / (2 eps)."""
    jp = misfit(c + eps * direction, omega, pml, F, receivers, data, C)
    jm = misfit(c - eps * direction, omega, pml, F, receivers, data, C)
    return (jp - jm) / (2.0 * eps)
