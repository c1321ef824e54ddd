"""The discrete PML Helmholtz operator A (Sec. 2.1, eq. helmd).

After dividing the stretched equation by s1 s2 it reads

  d1((s1/s2) d1 u) + d2((s2/s1) d2 u) + omega^2/(s1 s2 c^2) u = f,

and the 5-point stencil at p_{i,j} has the four neighbour coefficients

  W = (s1/s2)_{i-1/2,j}/h^2,  E = (s1/s2)_{i+1/2,j}/h^2,
  S = (s2/s1)_{i,j-1/2}/h^2,  N = (s2/s1)_{i,j+1/2}/h^2,

and the centre coefficient omega^2/((s1 s2)_{i,j} c_{i,j}^2) - (W+E+S+N).
Neighbours outside 1..n are zero (u = 0 on the boundary), but the centre
coefficient always subtracts all four.

Readings of the paper used here:
* (s1/s2)_{i+1/2,j} is s1 evaluated exactly at x_{i+1/2} divided by s2 at
  x_j (no averaging);
* every edge coefficient is computed once and used by both rows it couples,
  so A^t = A holds exactly (the paper's symmetry remark after eq. helmd);
* unknowns are ordered row by row, x1 index fastest: flat index
  (j-1) n + (i-1); layer m is grid row j = m.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .pml import DEFAULT_C, grid, stretch


@dataclass
class Stencil:
    n: int
    omega: float
    h: float
    W: np.ndarray   # (n, n) [j-1, i-1], coefficient of u_{i-1,j}
    E: np.ndarray   # coefficient of u_{i+1,j}
    S: np.ndarray   # coefficient of u_{i,j-1}
    N: np.ndarray   # coefficient of u_{i,j+1}
    D: np.ndarray   # centre coefficient
    s1s2: np.ndarray  # (s1 s2)_{i,j}, needed by the c-derivative of D
    c: np.ndarray


def stencil(c, omega, pml, C=DEFAULT_C):
    """Coefficient fields of eq. helmd for velocity c (shape (n, n))."""
    c = np.asarray(c, dtype=np.float64)
    n = c.shape[0]
    assert c.shape == (n, n)
    h, x, xh = grid(n)
    eta = pml * h
    s_node = stretch(x, omega, eta, C)
    s_half = stretch(xh, omega, eta, C)
    # Horizontal edge between (i, j) and (i+1, j), i = 0..n: (s1/s2)_{i+1/2, j}/h^2.
    ex = s_half[None, :] / s_node[:, None] / h ** 2           # (n, n+1), [j-1, i]
    # Vertical edge between (i, j) and (i, j+1), j = 0..n: (s2/s1)_{i, j+1/2}/h^2.
    ey = s_half[:, None] / s_node[None, :] / h ** 2           # (n+1, n), [j, i-1]
    W = ex[:, :n]
    E = ex[:, 1:]
    S = ey[:n, :]
    N = ey[1:, :]
    s1s2 = s_node[None, :] * s_node[:, None]
    D = omega ** 2 / (s1s2 * c ** 2) - (W + E + S + N)
    return Stencil(n=n, omega=omega, h=h, W=W, E=E, S=S, N=N, D=D, s1s2=s1s2, c=c)


def matrix(st: Stencil):
    """Sparse CSR matrix A of size n^2 with row (j-1) n + (i-1)."""
    n = st.n
    idx = np.arange(n * n).reshape(n, n)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [st.D.ravel()]
    # west / east neighbours (same row j)
    rows.append(idx[:, 1:].ravel()); cols.append(idx[:, :-1].ravel()); vals.append(st.W[:, 1:].ravel())
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel()); vals.append(st.E[:, :-1].ravel())
    # south / north neighbours (same column i)
    rows.append(idx[1:, :].ravel()); cols.append(idx[:-1, :].ravel()); vals.append(st.S[1:, :].ravel())
    rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel()); vals.append(st.N[:-1, :].ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n * n, n * n))
    return A.tocsr()


def apply(st: Stencil, u):
    """y = A u for u of shape (n*n,) or (k, n*n), without forming A."""
    n = st.n
    u = np.asarray(u)
    single = u.ndim == 1
    U = u.reshape(-1, n, n)
    Y = st.D[None] * U
    Y[:, :, 1:] += st.W[None, :, 1:] * U[:, :, :-1]
    Y[:, :, :-1] += st.E[None, :, :-1] * U[:, :, 1:]
    Y[:, 1:, :] += st.S[None, 1:, :] * U[:, :-1, :]
    Y[:, :-1, :] += st.N[None, :-1, :] * U[:, 1:, :]
    Y = Y.reshape(-1, n * n)
    return Y[0] if single else Y


def layer_blocks(st: Stencil, m):
    """Blocks of the layer-tridiagonal form for layer m (1-based).

    Returns (diag, upper) of the tridiagonal A_{m,m} (upper[i] couples i, i+1)
    and, for m > 1, the diagonal of A_{m,m-1} (= diagonal of A_{m-1,m}).
    """
    d = st.D[m - 1].copy()
    up = st.E[m - 1, :-1].copy()
    low = st.S[m - 1].copy() if m > 1 else None
    return d, up, low


def layer_tridiag(st: Stencil, m):
    d, up, _ = layer_blocks(st, m)
    lo = st.W[m - 1, 1:]
    return np.diag(d) + np.diag(up, 1) + np.diag(lo, -1)
