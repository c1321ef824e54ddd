"""Strongly admissible H-matrices, randomized SVD, and the approximate
sweeping factorization in that format (Sec. 2.3, strongly admissible case;
Sec. 2.4, Algs. 2.3 and 2.4).

TEST INFRASTRUCTURE ONLY (see the package docstring): plain recursive FP64
code, no blocking or fusion beyond what the operations state.

Format.  The index set 0..n-1 of a layer is bisected ([lo, mid), [mid, hi),
mid = lo + (hi - lo) // 2) to a fixed depth L, the smallest at which every
cluster holds at most `leaf` indices, so every leaf is on level L.  Two
clusters of one level are well separated when the distance between them is
at least their width: distance = min |p - q| over their indices, width = the
larger number of indices (each index owns one grid cell).  For clusters of
one level this holds exactly when at least one cluster lies between them.
A block (t, s) of two clusters of one level is

* 'F' (factorized, U V^t) when t and s are well separated -- its parent
  block was not, so s is in t's interaction list;
* 'D' (dense) when they are not and both are leaves;
* 'H' otherwise: the 2 x 2 blocks of the children.

So the diagonal and the blocks of adjacent clusters are refined down to the
leaves, and every block row carries up to three factorized blocks per level.

Operations, each recursive over this block tree:

* matvec / matvec_t -- G X and G^t X (hmatvec)
* add               -- hadd / hsub: F blocks concatenated and recompressed
                       (QR of both factors, truncated SVD of the small core)
* mul_add           -- T += alpha G H into the fixed block structure of T
                       (hmul).  A factorized operand makes the product low
                       rank, U (H^t V)^t or (G X) Y^t, which is added into T
                       along T's tree and recompressed in every F block it
                       lands on.  A dense target takes the dense product.  A
                       factorized target with two non-factorized operands is
                       the one new form, F = H . H, computed by randomized
                       SVD from products with Gaussian test vectors (two
                       hmatvecs per product).  Otherwise the three are split
                       into their children.
* inv               -- hinv: 2 x 2 block inversion through the Schur
                       complement of the first diagonal block
* diagmul_left/right -- hdiagmul

Truncation keeps sigma_k > tol * sigma_1 of each block (relative to that
block), at most rmax of them; tol = 0 and rmax = None truncate nothing.

Randomized SVD (Halko, Martinsson and Tropp, "Finding structure with
randomness", 2011: the range finder with Gaussian test matrix, then the
direct SVD of the projected matrix).  For an m x q product with l = min(k +
p, m, q) samples (k = rmax, or min(m, q) without truncation; p oversampling):
Y = (G H) Omega, Q = orth(Y), B = Q^H (G H) through (H^t (G^t conj(Q)))^t,
B = W S Z^H, and G H ~ (Q W_k S_k) (Z_k^H).  The Gaussian test matrices come
from the generator passed in.
"""
import numpy as np

from . import assemble
from .hmatrix import Trunc, compress
from .sweep import couplings

OVERSAMPLE = 8


# ----------------------------------------------------------------------------
# cluster tree and block structure

def depth(n, leaf):
    """Smallest L with every cluster of level L at most `leaf` indices."""
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    return L


def well_separated(t, s):
    """Clusters t = (lo, hi), s = (lo, hi): distance >= width."""
    if t[1] <= s[0]:
        dist = s[0] - (t[1] - 1)
    elif s[1] <= t[0]:
        dist = t[0] - (s[1] - 1)
    else:
        dist = 0
    return dist >= max(t[1] - t[0], s[1] - s[0])


def _split(c):
    lo, hi = c
    mid = lo + (hi - lo) // 2
    return (lo, mid), (mid, hi)


class SB:
    """A block of rows t and columns s (absolute index ranges) at `level`."""
    __slots__ = ("t", "s", "level", "kind", "d", "u", "v", "ch")

    def __init__(self, t, s, level, kind):
        self.t, self.s, self.level, self.kind = t, s, level, kind
        self.d = self.u = self.v = None
        self.ch = None

    @property
    def m(self):
        return self.t[1] - self.t[0]

    @property
    def q(self):
        return self.s[1] - self.s[0]

    def rows(self, child):
        """Slice of this block's rows that a child block covers."""
        return slice(child.t[0] - self.t[0], child.t[1] - self.t[0])

    def cols(self, child):
        return slice(child.s[0] - self.s[0], child.s[1] - self.s[0])


class Line:
    """Cluster geometry of a layer of a 2D grid: the indices 0..n-1 on a line,
    bisected; clusters are index ranges (lo, hi)."""

    def __init__(self, n, leaf):
        self.n = n
        self.L = depth(n, leaf)

    def root(self):
        return (0, self.n)

    def split(self, c):
        return _split(c)

    @staticmethod
    def rng(c):
        return c

    @staticmethod
    def admissible(t, s, level):
        return well_separated(t, s)


def structure(t, s, level, geo):
    """Zero block of the strong format on clusters t, s of one level."""
    tr, sr = geo.rng(t), geo.rng(s)
    if geo.admissible(t, s, level):
        b = SB(tr, sr, level, "F")
        b.u = np.zeros((b.m, 0), complex)
        b.v = np.zeros((b.q, 0), complex)
    elif level == geo.L:
        b = SB(tr, sr, level, "D")
        b.d = np.zeros((b.m, b.q), complex)
    else:
        b = SB(tr, sr, level, "H")
        tc, sc = geo.split(t), geo.split(s)
        b.ch = [[structure(tc[a], sc[c], level + 1, geo) for c in range(2)] for a in range(2)]
    return b


def zeros(n, leaf, geo=None):
    """The zero n x n matrix in the strong format (cluster geometry `geo`,
    by default the bisected line of n indices)."""
    geo = geo if geo is not None else Line(n, leaf)
    return structure(geo.root(), geo.root(), 0, geo)


def zeros_like(B):
    b = SB(B.t, B.s, B.level, B.kind)
    if B.kind == "F":
        b.u = np.zeros((B.m, 0), complex)
        b.v = np.zeros((B.q, 0), complex)
    elif B.kind == "D":
        b.d = np.zeros((B.m, B.q), complex)
    else:
        b.ch = [[zeros_like(B.ch[a][c]) for c in range(2)] for a in range(2)]
    return b


def blocks(B):
    """All leaves of the block tree (F and D blocks)."""
    if B.kind == "H":
        return [x for row in B.ch for c in row for x in blocks(c)]
    return [B]


# ----------------------------------------------------------------------------
# conversions and products with vectors

def from_dense(M, like, trunc):
    """M in the structure of `like`, F blocks by truncated SVD."""
    b = SB(like.t, like.s, like.level, like.kind)
    if like.kind == "D":
        b.d = np.array(M, dtype=complex)
    elif like.kind == "F":
        W, s, Zh = np.linalg.svd(M, full_matrices=False)
        k = trunc.keep(s)
        b.u, b.v = W[:, :k] * s[:k], Zh[:k].T
    else:
        b.ch = [[from_dense(M[like.rows(c)][:, like.cols(c)], c, trunc) for c in row] for row in like.ch]
    return b


def to_dense(B):
    if B.kind == "D":
        return B.d.copy()
    if B.kind == "F":
        return B.u @ B.v.T
    M = np.zeros((B.m, B.q), complex)
    for row in B.ch:
        for c in row:
            M[B.rows(c), B.cols(c)] = to_dense(c)
    return M


def matvec(B, X):
    """hmatvec: B X, X of shape (q,) or (q, k)."""
    if B.kind == "D":
        return B.d @ X
    if B.kind == "F":
        return B.u @ (B.v.T @ X)
    Y = np.zeros((B.m,) + X.shape[1:], complex)
    for row in B.ch:
        for c in row:
            Y[B.rows(c)] += matvec(c, X[B.cols(c)])
    return Y


def matvec_t(B, X):
    """B^t X, X of shape (m,) or (m, k)."""
    if B.kind == "D":
        return B.d.T @ X
    if B.kind == "F":
        return B.v @ (B.u.T @ X)
    Y = np.zeros((B.q,) + X.shape[1:], complex)
    for row in B.ch:
        for c in row:
            Y[B.cols(c)] += matvec_t(c, X[B.rows(c)])
    return Y


def max_rank(B):
    return max((b.u.shape[1] for b in blocks(B) if b.kind == "F"), default=0)


def storage(B):
    """Stored complex entries (dense leaves plus both factors of F blocks)."""
    return sum(b.d.size if b.kind == "D" else b.u.size + b.v.size for b in blocks(B))


# ----------------------------------------------------------------------------
# randomized SVD and the H-arithmetic

def rsvd(apply, apply_t, m, q, trunc, rng, oversample=OVERSAMPLE):
    """Low-rank U V^t of the m x q operator X -> apply(X) (apply_t(Y) is its
    transpose applied to Y), by the randomized range finder and a truncated
    SVD of the projected matrix."""
    k = trunc.rmax if trunc.rmax is not None else min(m, q)
    ell = min(k + oversample, m, q)
    if ell == 0:
        return np.zeros((m, 0), complex), np.zeros((q, 0), complex)
    omega = (rng.standard_normal((q, ell)) + 1j * rng.standard_normal((q, ell))) / np.sqrt(2.0)
    Q, _ = np.linalg.qr(apply(omega))
    B = apply_t(Q.conj()).T                       # Q^H (G H), ell x q
    W, s, Zh = np.linalg.svd(B, full_matrices=False)
    r = trunc.keep(s)
    return Q @ (W[:, :r] * s[:r]), Zh[:r].T


def add_lowrank(T, U, V, trunc):
    """T += U V^t along T's block tree, recompressing every F block."""
    if U.shape[1] == 0:
        return
    if T.kind == "D":
        T.d = T.d + U @ V.T
    elif T.kind == "F":
        T.u, T.v = compress(np.hstack([T.u, U]), np.hstack([T.v, V]), trunc)
    else:
        for row in T.ch:
            for c in row:
                add_lowrank(c, U[T.rows(c)], V[T.cols(c)], trunc)


def add(G, H, trunc, alpha=1.0):
    """hadd (alpha = 1) / hsub (alpha = -1) of two blocks of one structure."""
    b = SB(G.t, G.s, G.level, G.kind)
    if G.kind == "D":
        b.d = G.d + alpha * H.d
    elif G.kind == "F":
        b.u, b.v = compress(np.hstack([G.u, alpha * H.u]), np.hstack([G.v, H.v]), trunc)
    else:
        b.ch = [[add(G.ch[a][c], H.ch[a][c], trunc, alpha) for c in range(2)] for a in range(2)]
    return b


def mul_add(T, G, H, alpha, trunc, rng):
    """T += alpha G H, with G on (T's rows, u) and H on (u, T's columns),
    all three blocks of one level."""
    if G.kind == "F":                                       # F . X: U (X^t V)^t
        add_lowrank(T, alpha * G.u, matvec_t(H, G.v), trunc)
    elif H.kind == "F":                                     # X . F: (X U) V^t
        add_lowrank(T, alpha * matvec(G, H.u), H.v, trunc)
    elif T.kind == "D":                                     # dense leaves
        T.d = T.d + alpha * (G.d @ H.d)
    elif T.kind == "F":                                     # F = H . H
        U, V = rsvd(lambda X: matvec(G, matvec(H, X)), lambda Y: matvec_t(H, matvec_t(G, Y)),
                    T.m, T.q, trunc, rng)
        add_lowrank(T, alpha * U, V, trunc)
    else:
        for a in range(2):
            for c in range(2):
                for b in range(2):
                    mul_add(T.ch[a][c], G.ch[a][b], H.ch[b][c], alpha, trunc, rng)


def mul(G, H, like, trunc, rng, alpha=1.0):
    """hmul: alpha G H in the structure of `like`."""
    T = zeros_like(like)
    mul_add(T, G, H, alpha, trunc, rng)
    return T


def inv(G, trunc, rng):
    """hinv: with S = G22 - G21 G11^{-1} G12,
        G^{-1} = [[G11^{-1} + G11^{-1} G12 S^{-1} G21 G11^{-1}, -G11^{-1} G12 S^{-1}],
                  [-S^{-1} G21 G11^{-1},                          S^{-1}]].
    The diagonal blocks of the format are never factorized, so G is 'D' or
    'H'."""
    if G.kind == "D":
        b = SB(G.t, G.s, G.level, "D")
        b.d = np.linalg.inv(G.d)
        return b
    (G11, G12), (G21, G22) = G.ch
    Y = inv(G11, trunc, rng)                               # G11^{-1}
    Z = mul(Y, G12, G12, trunc, rng)                       # G11^{-1} G12
    X = mul(G21, Y, G21, trunc, rng)                       # G21 G11^{-1}
    S = add(G22, mul(G21, Z, G22, trunc, rng), trunc, alpha=-1.0)
    W = inv(S, trunc, rng)                                 # S^{-1}
    T12 = mul(Z, W, G12, trunc, rng, alpha=-1.0)           # -G11^{-1} G12 S^{-1}
    T21 = mul(W, X, G21, trunc, rng, alpha=-1.0)           # -S^{-1} G21 G11^{-1}
    T11 = add(Y, mul(Z, T21, G11, trunc, rng), trunc, alpha=-1.0)   # Y + Z S^{-1} X
    b = SB(G.t, G.s, G.level, "H")
    b.ch = [[T11, T12], [T21, W]]
    return b


def diagmul_left(d, B):
    """hdiagmul(D, B) = diag(d) B, d of length B.m."""
    b = SB(B.t, B.s, B.level, B.kind)
    if B.kind == "D":
        b.d = d[:, None] * B.d
    elif B.kind == "F":
        b.u, b.v = d[:, None] * B.u, B.v
    else:
        b.ch = [[diagmul_left(d[B.rows(c)], c) for c in row] for row in B.ch]
    return b


def diagmul_right(B, d):
    """hdiagmul(B, D) = B diag(d), d of length B.q."""
    b = SB(B.t, B.s, B.level, B.kind)
    if B.kind == "D":
        b.d = B.d * d[None, :]
    elif B.kind == "F":
        b.u, b.v = B.u, d[:, None] * B.v
    else:
        b.ch = [[diagmul_right(c, d[B.cols(c)]) for c in row] for row in B.ch]
    return b


# ----------------------------------------------------------------------------
# Alg. 2.3 and Alg. 2.4 in the strong format

def factor(st: assemble.Stencil, leaf, trunc, rng):
    """T~_1 = hinv(A_11); S~_m = hsub(A_mm, hdiagmul(A_{m,m-1}, hdiagmul(T~_{m-1},
    A_{m-1,m}))), T~_m = hinv(S~_m).  A_mm is tridiagonal, so all of it lies
    in the dense near-field blocks and its F blocks have rank 0."""
    n = st.n
    a = couplings(st)
    like = zeros(n, leaf)
    exact = Trunc()
    T = []
    for m in range(1, n + 1):
        d, up, _ = assemble.layer_blocks(st, m)
        lo = st.W[m - 1, 1:]
        Ad = np.diag(d.astype(complex)) + np.diag(up.astype(complex), 1) + np.diag(lo.astype(complex), -1)
        Ah = from_dense(Ad, like, exact)
        if m == 1:
            S = Ah
        else:
            am = a[m - 2]
            S = add(Ah, diagmul_left(am, diagmul_right(T[-1], am)), trunc, alpha=-1.0)
        T.append(inv(S, trunc, rng))
    return T


def solve(st: assemble.Stencil, T, f):
    """Alg. 2.4: the sweep with hmatvec(T~_m, .) in the strong format."""
    n = st.n
    a = couplings(st)
    f = np.asarray(f, dtype=np.complex128)
    single = f.ndim == 1
    F = f.reshape(-1, n, n)
    out = np.empty_like(F)
    for k in range(F.shape[0]):
        u = F[k].copy()
        w = np.empty_like(u)
        for m in range(n):
            if m > 0:
                u[m] = u[m] - a[m - 1] * w[m - 1]
            w[m] = matvec(T[m], u[m])
        u[n - 1] = w[n - 1]
        for m in range(n - 2, -1, -1):
            u[m] = w[m] - matvec(T[m], a[m] * u[m + 1])
        out[k] = u
    out = out.reshape(-1, n * n)
    return out[0] if single else out
