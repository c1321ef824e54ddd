"""The 3D method (Sec. 4): the 7-point PML operator, the face-by-face
sweeping factorization with exact (dense) face Schur complements, and the
approximate one with strongly admissible H-matrices on the faces.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Operator (Sec. 4, discretization).  With s_a = (1 + i sigma(x_a)/omega)^{-1}
on each axis, the equation divided by s1 s2 s3 reads
  d1((s1/(s2 s3)) d1 u) + d2((s2/(s1 s3)) d2 u) + d3((s3/(s1 s2)) d3 u)
    + omega^2/(s1 s2 s3 c^2) u = f,
and the 7-point stencil at p_{i,j,k} couples to its six neighbours with the
coefficient of that edge, e.g. (s1/(s2 s3))_{i+1/2,j,k}/h^2 towards p_{i+1,j,k};
the centre coefficient is omega^2/((s1 s2 s3)_{i,j,k} c^2) minus all six.
As in 2D, s_a is evaluated exactly at nodes and half nodes and each edge
coefficient is computed once for both rows it couples (A = A^t bitwise).
Unknowns are ordered x1 fastest, then x2, then x3: flat index
(k-1) n^2 + (j-1) n + (i-1); face m is the plane x3 = m h, and A is block
tridiagonal in the faces with diagonal couplings A_{m,m-1} = A_{m-1,m}^t.

Exact sweep.  T_1 = A_{1,1}^{-1}, T_m = (A_{m,m} - A_{m,m-1} T_{m-1} A_{m-1,m})^{-1}
with dense n^2 x n^2 faces, then the sweep of Alg. 2.2 face by face.

Face H-matrices (Sec. 4, hierarchical matrix representation).  The points of
a face are clustered by bisection in both x1 and x2: quadtree level l has
2^l x 2^l boxes.  Two boxes (i, j), (i', j') of one level are well separated
when max(|i - i'|, |j - j'|) > 1 (strong admissibility), and a block is
factorized when its boxes are well separated but their parents are not.
Reading: one quadtree level is taken as two bisections, first in x1 and then
in x2, so that the 2 x 2 block inversion of hinv applies; admissibility is
tested on the quadtree levels only (the half boxes in between are always
refined), which gives exactly the quadtree block partition.  The face
points are ordered by this recursive bisection so that every cluster is a
contiguous index range; the strong format and its arithmetic (oracle.strong)
then apply unchanged, with this cluster geometry.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import strong
from .hmatrix import Trunc
from .pml import DEFAULT_C, grid, stretch_sides


@dataclass
class Stencil3:
    n: int
    omega: float
    h: float
    X0: np.ndarray   # (n, n, n) [k-1, j-1, i-1]: coefficient of u_{i-1,j,k}
    X1: np.ndarray   # u_{i+1,j,k}
    Y0: np.ndarray   # u_{i,j-1,k}
    Y1: np.ndarray   # u_{i,j+1,k}
    Z0: np.ndarray   # u_{i,j,k-1}
    Z1: np.ndarray   # u_{i,j,k+1}
    D: np.ndarray    # centre
    s123: np.ndarray
    c: np.ndarray


def widths3(pml):
    """(x1 lo, x1 hi, x2 lo, x2 hi, x3 lo, x3 hi) from one width or six."""
    if np.isscalar(pml):
        return (int(pml),) * 6
    w = tuple(int(v) for v in pml)
    assert len(w) == 6
    return w


def stencil(c, omega, pml, C=DEFAULT_C):
    """Coefficient fields for velocity c of shape (n, n, n), indexed [k, j, i]."""
    c = np.asarray(c, dtype=np.float64)
    n = c.shape[0]
    assert c.shape == (n, n, n)
    h, x, xh = grid(n)
    w = widths3(pml)
    s_node = [stretch_sides(x, omega, w[2 * a] * h, w[2 * a + 1] * h, C) for a in range(3)]
    s_half = [stretch_sides(xh, omega, w[2 * a] * h, w[2 * a + 1] * h, C) for a in range(3)]
    s1, s2, s3 = s_node
    # edge between (i, j, k) and (i+1, j, k) at half index ih = 0..n: (s1/(s2 s3))_{ih - 1/2} / h^2
    ex = s_half[0][None, None, :] / (s2[None, :, None] * s3[:, None, None]) / h ** 2      # (n, n, n+1)
    ey = s_half[1][None, :, None] / (s1[None, None, :] * s3[:, None, None]) / h ** 2      # (n, n+1, n)
    ez = s_half[2][:, None, None] / (s1[None, None, :] * s2[None, :, None]) / h ** 2      # (n+1, n, n)
    X0, X1 = ex[:, :, :n].copy(), ex[:, :, 1:].copy()
    Y0, Y1 = ey[:, :n, :].copy(), ey[:, 1:, :].copy()
    Z0, Z1 = ez[:n].copy(), ez[1:].copy()
    s123 = s1[None, None, :] * s2[None, :, None] * s3[:, None, None]
    D = omega ** 2 / (s123 * c ** 2) - (X0 + X1 + Y0 + Y1 + Z0 + Z1)
    return Stencil3(n=n, omega=omega, h=h, X0=X0, X1=X1, Y0=Y0, Y1=Y1, Z0=Z0, Z1=Z1, D=D, s123=s123, c=c)


def matrix(st: Stencil3):
    """Sparse CSR A of size n^3, row (k-1) n^2 + (j-1) n + (i-1)."""
    n = st.n
    idx = np.arange(n ** 3).reshape(n, n, n)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [st.D.ravel()]

    def add(sl_to, sl_from, coef):
        rows.append(idx[sl_to].ravel())
        cols.append(idx[sl_from].ravel())
        vals.append(coef[sl_to].ravel())
    a, b = slice(1, None), slice(None, -1)
    full = slice(None)
    add((full, full, a), (full, full, b), st.X0)
    add((full, full, b), (full, full, a), st.X1)
    add((full, a, full), (full, b, full), st.Y0)
    add((full, b, full), (full, a, full), st.Y1)
    add((a, full, full), (b, full, full), st.Z0)
    add((b, full, full), (a, full, full), st.Z1)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n ** 3, n ** 3))
    return A.tocsr()


def apply(st: Stencil3, u):
    """y = A u for u of shape (n^3,) or (r, n^3)."""
    n = st.n
    u = np.asarray(u)
    single = u.ndim == 1
    U = u.reshape(-1, n, n, n)
    Y = st.D[None] * U
    Y[..., 1:] += st.X0[None, :, :, 1:] * U[..., :-1]
    Y[..., :-1] += st.X1[None, :, :, :-1] * U[..., 1:]
    Y[:, :, 1:, :] += st.Y0[None, :, 1:, :] * U[:, :, :-1, :]
    Y[:, :, :-1, :] += st.Y1[None, :, :-1, :] * U[:, :, 1:, :]
    Y[:, 1:] += st.Z0[None, 1:] * U[:, :-1]
    Y[:, :-1] += st.Z1[None, :-1] * U[:, 1:]
    Y = Y.reshape(-1, n ** 3)
    return Y[0] if single else Y


def face_operator(st: Stencil3, m):
    """Dense A_{m,m} (n^2 x n^2, face points x1 fastest) of face m (0-based)."""
    n = st.n
    idx = np.arange(n * n).reshape(n, n)
    A = np.zeros((n * n, n * n), dtype=np.complex128)
    A[idx.ravel(), idx.ravel()] = st.D[m].ravel()
    A[idx[:, 1:].ravel(), idx[:, :-1].ravel()] = st.X0[m][:, 1:].ravel()
    A[idx[:, :-1].ravel(), idx[:, 1:].ravel()] = st.X1[m][:, :-1].ravel()
    A[idx[1:, :].ravel(), idx[:-1, :].ravel()] = st.Y0[m][1:, :].ravel()
    A[idx[:-1, :].ravel(), idx[1:, :].ravel()] = st.Y1[m][:-1, :].ravel()
    return A


def face_couplings(st: Stencil3):
    """a[m] = diagonal of A_{m+1,m} (0-based faces m = 0..n-2), shape (n-1, n^2)."""
    return st.Z0[1:].reshape(st.n - 1, -1).copy()


# ----------------------------------------------------------------------------
# separable closed form (c constant)

def _operator_1d(n, omega, lo, hi, C):
    h, x, xh = grid(n)
    s = stretch_sides(x, omega, lo * h, hi * h, C)
    sh = stretch_sides(xh, omega, lo * h, hi * h, C)
    L = np.zeros((n, n), dtype=np.complex128)
    i = np.arange(n)
    L[i, i] = -s * (sh[:-1] + sh[1:]) / h ** 2
    L[i[1:], i[1:] - 1] = s[1:] * sh[1:-1] / h ** 2
    L[i[:-1], i[:-1] + 1] = s[:-1] * sh[1:-1] / h ** 2
    return L, s


def solve_constant(n, omega, pml, c0, f, C=DEFAULT_C):
    """A u = f for c = c0 by fast diagonalization: multiplying row (i, j, k) by
    (s1 s2 s3)_{i,j,k} gives the Kronecker sum (L1 + L2 + L3 + omega^2/c0^2) u
    = (s1 s2 s3) f of the 1D operators (L v)_i = s_i [s_{i-1/2}(v_{i-1} - v_i) +
    s_{i+1/2}(v_{i+1} - v_i)]/h^2, solved in the eigenbases of L1, L2, L3
    (Lynch, Rice and Thomas).  Built from the 1D factors only."""
    w = widths3(pml)
    Ls = [_operator_1d(n, omega, w[2 * a], w[2 * a + 1], C) for a in range(3)]
    eig = [np.linalg.eig(L) for L, _ in Ls]
    lam = [e[0] for e in eig]
    V = [e[1] for e in eig]
    Vi = [np.linalg.inv(v) for v in V]
    s1, s2, s3 = (Ls[a][1] for a in range(3))
    G = (s3[:, None, None] * s2[None, :, None] * s1[None, None, :]) * np.asarray(f, np.complex128).reshape(n, n, n)
    def along(M, X):                       # apply M along x1, x2, x3 in turn: [k, j, i] fields
        M1, M2, M3 = M
        X = X @ M1.T
        X = np.einsum("jb,kbi->kji", M2, X)
        return np.einsum("kc,cji->kji", M3, X)
    Gt = along(Vi, G)
    Ut = Gt / (lam[2][:, None, None] + lam[1][None, :, None] + lam[0][None, None, :] + omega ** 2 / c0 ** 2)
    return along(V, Ut).reshape(-1)


# ----------------------------------------------------------------------------
# exact face-by-face sweep (Algs. 2.1 and 2.2 in 3D)

def factor_exact(st: Stencil3):
    n = st.n
    a = face_couplings(st)
    T = []
    for m in range(n):
        S = face_operator(st, m)
        if m > 0:
            S = S - (a[m - 1][:, None] * T[-1]) * a[m - 1][None, :]
        T.append(np.linalg.inv(S))
    return T


def _sweep(st: Stencil3, f, apply_T):
    n = st.n
    N2 = n * n
    a = face_couplings(st)
    f = np.asarray(f, dtype=np.complex128)
    single = f.ndim == 1
    F = f.reshape(-1, n, N2)
    out = np.empty_like(F)
    for r in range(F.shape[0]):
        u = F[r].copy()
        w = np.empty_like(u)
        for m in range(n):
            if m > 0:
                u[m] = u[m] - a[m - 1] * w[m - 1]
            w[m] = apply_T(m, u[m])
        u[n - 1] = w[n - 1]
        for m in range(n - 2, -1, -1):
            u[m] = w[m] - apply_T(m, a[m] * u[m + 1])
        out[r] = u
    out = out.reshape(-1, n ** 3)
    return out[0] if single else out


def solve_exact(st: Stencil3, T, f):
    return _sweep(st, f, lambda m, v: T[m] @ v)


# ----------------------------------------------------------------------------
# face H-matrices: cluster geometry, factorization and sweep

class Face:
    """Cluster geometry of an n x n face for oracle.strong: clusters are boxes
    (i0, i1, j0, j1) of face points, bisected in x1 on even binary levels and
    in x2 on odd ones, each a contiguous range of `perm` (the face points in
    bisection order).  Quadtree level l is binary level 2 l."""

    def __init__(self, n, leaf):
        self.n = n
        Lq = 0
        while (-(-n // (1 << Lq))) ** 2 > leaf:
            Lq += 1
        self.L = 2 * Lq
        order = []
        self._collect((0, n, 0, n), 0, order)
        self.perm = np.array(order)                     # bisection position -> natural face index

    def _collect(self, box, lev, out):
        if lev == self.L:
            i0, i1, j0, j1 = box
            out.extend(j * self.n + i for j in range(j0, j1) for i in range(i0, i1))
            return
        for b in self._halves(box, lev):
            self._collect(b, lev + 1, out)

    @staticmethod
    def _halves(box, lev):
        i0, i1, j0, j1 = box
        if lev % 2 == 0:
            mid = i0 + (i1 - i0) // 2
            return (i0, mid, j0, j1), (mid, i1, j0, j1)
        mid = j0 + (j1 - j0) // 2
        return (i0, i1, j0, mid), (i0, i1, mid, j1)

    # a cluster: (lo, hi, box, binary level, quadtree coordinates (qi, qj))
    def root(self):
        return (0, self.n * self.n, (0, self.n, 0, self.n), 0, (0, 0))

    def split(self, c):
        lo, hi, box, lev, (qi, qj) = c
        b1, b2 = self._halves(box, lev)
        size1 = (b1[1] - b1[0]) * (b1[3] - b1[2])
        if lev % 2 == 0:
            q1, q2 = (2 * qi, qj), (2 * qi + 1, qj)
        else:
            q1, q2 = (qi, 2 * qj), (qi, 2 * qj + 1)
        return (lo, lo + size1, b1, lev + 1, q1), (lo + size1, hi, b2, lev + 1, q2)

    @staticmethod
    def rng(c):
        return (c[0], c[1])

    @staticmethod
    def admissible(t, s, level):
        if level % 2:
            return False
        (ti, tj), (si, sj) = t[4], s[4]
        return max(abs(ti - si), abs(tj - sj)) > 1


def factor_strong(st: Stencil3, leaf, trunc, rng):
    """Alg. 2.3 face by face with strongly admissible face H-matrices, in the
    bisection order of the face points: S~_1 = A_11, S~_m = hsub(A_mm,
    hdiagmul(A_{m,m-1}, hdiagmul(T~_{m-1}, A_{m-1,m}))), T~_m = hinv(S~_m).
    Returns (T~, face geometry)."""
    n = st.n
    geo = Face(n, leaf)
    P = geo.perm
    like = strong.zeros(n * n, leaf, geo)
    a = face_couplings(st)[:, P]
    exact = Trunc()
    T = []
    for m in range(n):
        Ap = face_operator(st, m)[np.ix_(P, P)]
        Ah = strong.from_dense(Ap, like, exact)
        if m == 0:
            S = Ah
        else:
            S = strong.add(Ah, strong.diagmul_left(a[m - 1], strong.diagmul_right(T[-1], a[m - 1])), trunc,
                           alpha=-1.0)
        T.append(strong.inv(S, trunc, rng))
    return T, geo


def solve_strong(st: Stencil3, T, geo, f):
    """Alg. 2.4 in 3D: the sweep with hmatvec of the face H-matrices (the
    fields are permuted into bisection order face by face and back)."""
    P = geo.perm
    inv = np.empty_like(P)
    inv[P] = np.arange(P.size)
    return _sweep(st, f, lambda m, v: strong.matvec(T[m], v[P])[inv])
