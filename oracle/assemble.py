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

from .pml import DEFAULT_C, grid, stretch_sides


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


def pml_widths(pml):
    """(x1 low, x1 high, x2 low, x2 high) widths in grid points from one width
    for every side or a 4-tuple."""
    if np.isscalar(pml):
        return (int(pml),) * 4
    w = tuple(int(v) for v in pml)
    assert len(w) == 4
    return w


def stencil(c, omega, pml, C=DEFAULT_C, abc=()):
    """Coefficient fields of eq. helmd for velocity c (shape (n, n)).

    pml: the absorbing-layer width in grid points on every side, or the
    widths (x1 low, x1 high, x2 low, x2 high); s1 is built from the x1 pair
    and s2 from the x2 pair.  abc: edges (names from EDGES) that carry the
    second-order absorbing boundary condition instead of u = 0; their layer
    width must be 0 (see `absorbing_closure`)."""
    c = np.asarray(c, dtype=np.float64)
    n = c.shape[0]
    assert c.shape == (n, n)
    h, x, xh = grid(n)
    a1, b1, a2, b2 = pml_widths(pml)
    s1_node = stretch_sides(x, omega, a1 * h, b1 * h, C)
    s1_half = stretch_sides(xh, omega, a1 * h, b1 * h, C)
    s2_node = stretch_sides(x, omega, a2 * h, b2 * h, C)
    s2_half = stretch_sides(xh, omega, a2 * h, b2 * h, C)
    # Horizontal edge between (i, j) and (i+1, j), i = 0..n: (s1/s2)_{i+1/2, j}/h^2.
    ex = s1_half[None, :] / s2_node[:, None] / h ** 2         # (n, n+1), [j-1, i]
    # Vertical edge between (i, j) and (i, j+1), j = 0..n: (s2/s1)_{i, j+1/2}/h^2.
    ey = s2_half[:, None] / s1_node[None, :] / h ** 2         # (n+1, n), [j, i-1]
    W = ex[:, :n]
    E = ex[:, 1:]
    S = ey[:n, :]
    N = ey[1:, :]
    s1s2 = s1_node[None, :] * s2_node[:, None]
    D = omega ** 2 / (s1s2 * c ** 2) - (W + E + S + N)
    st = Stencil(n=n, omega=omega, h=h, W=W.copy(), E=E.copy(), S=S.copy(), N=N.copy(), D=D, s1s2=s1s2, c=c)
    if abc:
        widths = dict(zip(EDGES, (a1, b1, a2, b2)))
        for e in abc:
            assert e in EDGES and widths[e] == 0, "an absorbing-condition edge has no layer"
        absorbing_closure(st, tuple(abc))
    return st


def abc_a(k, h):
    """u_b = a u_0 + g D_tt u_0: the weight of u_0 (see absorbing_closure)."""
    return (2 + 1j * k * h) / (2 - 1j * k * h)


def abc_g(k, h):
    """The weight of the tangential second difference (see absorbing_closure)."""
    return 1j * h / (k * (2 - 1j * k * h))


def absorbing_closure(st: Stencil, abc):
    """Second-order absorbing boundary condition (Sec. 3, other boundary
    conditions; Engquist and Majda) on the edges in `abc`, in place.

    On an edge with outward normal n and tangent t the condition is
        du/dn = i k u + (i / (2k)) d2u/dt2,   k = omega / c,
    which a plane wave leaving the domain at angle theta meets up to
    O(theta^4).  It is imposed at the half point between the boundary node
    u_b and the first interior node u_0 of each line normal to the edge:
        (u_b - u_0)/h = i k (u_b + u_0)/2 + (i/(2k)) D_tt u_0,
    D_tt the second difference along the edge, so that
        u_b = a u_0 + g D_tt u_0,  a = (2 + i k h)/(2 - i k h),  g = i h / (k (2 - i k h)),
    and u_b is eliminated from the row of u_0: its coefficient e_b (the
    edge coupling to the boundary node) moves e_b a onto the diagonal and
    e_b g D_tt u_0 into couplings along the edge.  Those are written in flux
    form with one weight per edge, tau = (w_p + w_q)/2 with w = e_b g / h^2
    at each of its two points, so the operator stays symmetric.  At an end
    of the edge the flux goes to the corner value: zero where the adjacent
    side is not absorbing (its boundary value is zero), none where it is.
    The edge couplings to the boundary nodes themselves stay in W/E/S/N."""
    n, h, om = st.n, st.h, st.omega
    k_of = lambda cv: om / cv                     # noqa: E731
    for e in abc:
        if e in ("x1=0", "x1=1"):
            col = 0 if e == "x1=0" else n - 1
            eb = (st.W[:, 0] if e == "x1=0" else st.E[:, n - 1]).copy()
            k = k_of(st.c[:, col])
            st.D[:, col] += eb * abc_a(k, h)
            w = eb * abc_g(k, h) / h ** 2
            tau = 0.5 * (w[:-1] + w[1:])                 # edge between rows j and j+1
            st.N[:-1, col] += tau
            st.S[1:, col] += tau
            st.D[:-1, col] -= tau
            st.D[1:, col] -= tau
            if "x2=0" not in abc:
                st.D[0, col] -= w[0]
            if "x2=1" not in abc:
                st.D[n - 1, col] -= w[n - 1]
        else:
            row = 0 if e == "x2=0" else n - 1
            eb = (st.S[0, :] if e == "x2=0" else st.N[n - 1, :]).copy()
            k = k_of(st.c[row, :])
            st.D[row, :] += eb * abc_a(k, h)
            w = eb * abc_g(k, h) / h ** 2
            tau = 0.5 * (w[:-1] + w[1:])                 # edge between columns i and i+1
            st.E[row, :-1] += tau
            st.W[row, 1:] += tau
            st.D[row, :-1] -= tau
            st.D[row, 1:] -= tau
            if "x1=0" not in abc:
                st.D[row, 0] -= w[0]
            if "x1=1" not in abc:
                st.D[row, n - 1] -= w[n - 1]


# The four edges of the unit square, for Dirichlet data u = b on an edge.
EDGES = ("x1=0", "x1=1", "x2=0", "x2=1")


def dirichlet_forcing(st: Stencil, edge, b):
    """The right-hand side term of Dirichlet data u = b on one edge (Sec. 2.5,
    depth extrapolation: the boundary values become a forcing on the layer of
    unknowns next to that edge).  Row p next to the edge has the coefficient
    of its boundary neighbour in W, E, S or N; moving that term to the right
    side gives -coefficient * b.  b: n values along the edge (index i-1 or
    j-1), or (k, n) for k right-hand sides.  Returns (n*n,) or (k, n*n)."""
    n = st.n
    b = np.asarray(b, dtype=np.complex128)
    single = b.ndim == 1
    B = b.reshape(-1, n)
    G = np.zeros((B.shape[0], n, n), dtype=np.complex128)
    if edge == "x2=1":
        G[:, n - 1, :] = -st.N[n - 1][None, :] * B
    elif edge == "x2=0":
        G[:, 0, :] = -st.S[0][None, :] * B
    elif edge == "x1=0":
        G[:, :, 0] = -st.W[:, 0][None, :] * B
    elif edge == "x1=1":
        G[:, :, n - 1] = -st.E[:, n - 1][None, :] * B
    else:
        raise ValueError(edge)
    G = G.reshape(-1, n * n)
    return G[0] if single else G


# Sweep directions (Sec. 2.4): the layers are rows swept upward (+x2) or
# downward (-x2), or columns swept rightward (+x1) or leftward (-x1).  A
# direction is a relabelling of the grid, frame point (i', m') <- natural
# point (i, j); sweeping the relabelled operator upward is sweeping the
# original one in that direction.
DIRECTIONS = ("+x2", "-x2", "+x1", "-x1")


def to_frame(field, direction):
    """A field indexed [j, i] (natural) as [m', i'] (frame of the direction)."""
    F = np.asarray(field)
    if direction == "+x2":
        return F
    if direction == "-x2":
        return F[..., ::-1, :]
    if direction == "+x1":
        return np.swapaxes(F, -1, -2)
    if direction == "-x1":
        return np.swapaxes(F, -1, -2)[..., ::-1, :]
    raise ValueError(direction)


def from_frame(field, direction):
    F = np.asarray(field)
    if direction in ("+x2", "+x1"):
        return to_frame(F, direction)
    if direction == "-x2":
        return F[..., ::-1, :]
    if direction == "-x1":
        return np.swapaxes(F[..., ::-1, :], -1, -2)
    raise ValueError(direction)


def permuted(st: Stencil, direction):
    """The stencil of the relabelled grid: the coefficient towards each frame
    neighbour is the natural coefficient towards the same grid point."""
    tf = lambda a: np.ascontiguousarray(to_frame(a, direction))  # noqa: E731
    if direction == "+x2":
        W, E, S, N = st.W, st.E, st.S, st.N
    elif direction == "-x2":       # frame layer m'+1 is the natural row below
        W, E, S, N = tf(st.W), tf(st.E), tf(st.N), tf(st.S)
    elif direction == "+x1":       # frame rows run along x2, layers are columns
        W, E, S, N = tf(st.S), tf(st.N), tf(st.W), tf(st.E)
    elif direction == "-x1":       # columns swept leftward
        W, E, S, N = tf(st.S), tf(st.N), tf(st.E), tf(st.W)
    else:
        raise ValueError(direction)
    return Stencil(n=st.n, omega=st.omega, h=st.h, W=W, E=E, S=S, N=N, D=tf(st.D), s1s2=tf(st.s1s2), c=tf(st.c))


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
