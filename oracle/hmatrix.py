"""Weakly admissible H-matrices and the approximate sweeping factorization.

Follows Sec. 2.3 (hierarchical matrix representation, weakly admissible
case) and Sec. 2.4 (Algs. 2.3 and 2.4) step by step, recursively, in FP64:

* the index set of a layer is bisected until a block holds at most
  `leaf` indices; the two off-diagonal blocks of every split are stored as
  U V^t, the diagonal blocks recursively, the finest ones densely;
* hmatvec   -- off-diagonal blocks as U (V^t f), diagonal blocks recursive;
* hadd/hsub -- blockwise; off-diagonal factors are concatenated and
               recompressed by QR of both factors and a truncated SVD of
               the small core;
* hmul      -- off-diagonal blocks through H x (low rank) products, which
               are matrix-vector products; diagonal blocks recursively plus
               the low-rank x low-rank term (middle product first), then
               hadd;
* hinv      -- 2 x 2 block inversion with the Schur complement
               S = G22 - G21 G11^{-1} G12, both inverses recursive;
* hdiagmul  -- scaling of U rows (left) or V rows (right), recursive.

Truncation keeps the singular values sigma_k > tol * sigma_1 of each
recompressed block (relative to that block), at most `rmax` of them;
tol = 0 and rmax = None disable truncation, and then every operation is
exact up to rounding.

The index set is split as [0, n//2) and [n//2, n), so sizes that are not
powers of two are bisected unevenly.
"""
import numpy as np

from . import assemble
from .sweep import couplings


class Trunc:
    def __init__(self, tol=0.0, rmax=None):
        self.tol = float(tol)
        self.rmax = rmax

    def keep(self, s):
        if s.size == 0 or s[0] == 0:
            return 0
        k = int(np.sum(s > self.tol * s[0])) if self.tol > 0 else int(np.sum(s > 0))
        if self.rmax is not None:
            k = min(k, self.rmax)
        return k


class HM:
    """Either a dense leaf (`d`) or a 2 x 2 split with low-rank off-diagonals."""
    __slots__ = ("n", "d", "a11", "a22", "u12", "v12", "u21", "v21")

    def __init__(self, n, d=None, a11=None, a22=None, u12=None, v12=None, u21=None, v21=None):
        self.n = n
        self.d = d
        self.a11, self.a22 = a11, a22
        self.u12, self.v12, self.u21, self.v21 = u12, v12, u21, v21

    @property
    def leaf(self):
        return self.d is not None

    @property
    def n1(self):
        return self.n // 2


def compress(U, V, trunc):
    """Truncated U V^t through QR of both factors and SVD of the core."""
    p, q = U.shape[0], V.shape[0]
    if U.shape[1] == 0:
        return np.zeros((p, 0), complex), np.zeros((q, 0), complex)
    Q1, R1 = np.linalg.qr(U)
    Q2, R2 = np.linalg.qr(V)
    W, s, Zh = np.linalg.svd(R1 @ R2.T)
    k = trunc.keep(s)
    return Q1 @ (W[:, :k] * s[:k]), Q2 @ Zh[:k].T


def tridiag(d, up, lo, leaf):
    """H-form of a tridiagonal matrix (diag d, superdiag up, subdiag lo)."""
    n = d.size
    if n <= leaf:
        return HM(n, d=np.diag(d) + np.diag(up, 1) + np.diag(lo, -1))
    n1 = n // 2
    e1 = np.zeros((n1, 1), complex)
    e2 = np.zeros((n - n1, 1), complex)
    e1[-1, 0] = 1.0
    e2[0, 0] = 1.0
    return HM(n,
              a11=tridiag(d[:n1], up[:n1 - 1], lo[:n1 - 1], leaf),
              a22=tridiag(d[n1:], up[n1:], lo[n1:], leaf),
              u12=e1 * up[n1 - 1], v12=e2.copy(),
              u21=e2 * lo[n1 - 1], v21=e1.copy())


def from_dense(M, leaf, trunc):
    n = M.shape[0]
    if n <= leaf:
        return HM(n, d=np.array(M, dtype=complex))
    n1 = n // 2
    W, s, Zh = np.linalg.svd(M[:n1, n1:])
    k = trunc.keep(s)
    W2, s2, Zh2 = np.linalg.svd(M[n1:, :n1])
    k2 = trunc.keep(s2)
    return HM(n, a11=from_dense(M[:n1, :n1], leaf, trunc), a22=from_dense(M[n1:, n1:], leaf, trunc),
              u12=W[:, :k] * s[:k], v12=Zh[:k].T, u21=W2[:, :k2] * s2[:k2], v21=Zh2[:k2].T)


def to_dense(G):
    if G.leaf:
        return G.d.copy()
    n1 = G.n1
    M = np.zeros((G.n, G.n), complex)
    M[:n1, :n1] = to_dense(G.a11)
    M[n1:, n1:] = to_dense(G.a22)
    M[:n1, n1:] = G.u12 @ G.v12.T
    M[n1:, :n1] = G.u21 @ G.v21.T
    return M


def matvec(G, X):
    """hmatvec: G X for X of shape (n,) or (n, k)."""
    if G.leaf:
        return G.d @ X
    n1 = G.n1
    X1, X2 = X[:n1], X[n1:]
    y1 = matvec(G.a11, X1) + G.u12 @ (G.v12.T @ X2)
    y2 = G.u21 @ (G.v21.T @ X1) + matvec(G.a22, X2)
    return np.concatenate([y1, y2], axis=0)


def matvec_t(G, X):
    """G^t X, recursing through the transposed blocks."""
    if G.leaf:
        return G.d.T @ X
    n1 = G.n1
    X1, X2 = X[:n1], X[n1:]
    y1 = matvec_t(G.a11, X1) + G.v21 @ (G.u21.T @ X2)
    y2 = G.v12 @ (G.u12.T @ X1) + matvec_t(G.a22, X2)
    return np.concatenate([y1, y2], axis=0)


def lowrank_like(P, Q, like):
    """P Q^t written in the block structure of `like` (no truncation needed)."""
    if like.leaf:
        return HM(like.n, d=P @ Q.T)
    n1 = like.n1
    return HM(like.n,
              a11=lowrank_like(P[:n1], Q[:n1], like.a11),
              a22=lowrank_like(P[n1:], Q[n1:], like.a22),
              u12=P[:n1], v12=Q[n1:], u21=P[n1:], v21=Q[:n1])


def add(G, H, trunc, alpha=1.0):
    """hadd (alpha = 1) / hsub (alpha = -1): G + alpha H, recompressed."""
    if G.leaf:
        return HM(G.n, d=G.d + alpha * H.d)
    u12, v12 = compress(np.hstack([G.u12, alpha * H.u12]), np.hstack([G.v12, H.v12]), trunc)
    u21, v21 = compress(np.hstack([G.u21, alpha * H.u21]), np.hstack([G.v21, H.v21]), trunc)
    return HM(G.n, a11=add(G.a11, H.a11, trunc, alpha), a22=add(G.a22, H.a22, trunc, alpha),
              u12=u12, v12=v12, u21=u21, v21=v21)


def mul(G, H, trunc):
    """hmul: G H in H-form."""
    if G.leaf:
        return HM(G.n, d=G.d @ H.d)
    # off-diagonal (1,2): G11 H12 + G12 H22 = (G11 X12) Y12^t + U12 (H22^t V12)^t
    u12, v12 = compress(np.hstack([matvec(G.a11, H.u12), G.u12]),
                        np.hstack([H.v12, matvec_t(H.a22, G.v12)]), trunc)
    # off-diagonal (2,1): G21 H11 + G22 H21 = U21 (H11^t V21)^t + (G22 X21) Y21^t
    u21, v21 = compress(np.hstack([G.u21, matvec(G.a22, H.u21)]),
                        np.hstack([matvec_t(H.a11, G.v21), H.v21]), trunc)
    # diagonal (1,1): G11 H11 + U12 (V12^t X21) Y21^t
    a11 = add(mul(G.a11, H.a11, trunc),
              lowrank_like(G.u12 @ (G.v12.T @ H.u21), H.v21, G.a11), trunc)
    # diagonal (2,2): U21 (V21^t X12) Y12^t + G22 H22
    a22 = add(mul(G.a22, H.a22, trunc),
              lowrank_like(G.u21 @ (G.v21.T @ H.u12), H.v12, G.a22), trunc)
    return HM(G.n, a11=a11, a22=a22, u12=u12, v12=v12, u21=u21, v21=v21)


def inv(G, trunc):
    """hinv: 2 x 2 block inverse through the Schur complement of G11."""
    if G.leaf:
        return HM(G.n, d=np.linalg.inv(G.d))
    A = inv(G.a11, trunc)                                  # G11^{-1}
    AU = matvec(A, G.u12)                                  # G11^{-1} U12
    core = G.v21.T @ AU                                    # V21^t G11^{-1} U12
    S = add(G.a22, lowrank_like(G.u21 @ core, G.v12, G.a22), trunc, alpha=-1.0)
    Si = inv(S, trunc)                                     # S^{-1}
    SiU = matvec(Si, G.u21)                                # S^{-1} U21
    ATV = matvec_t(A, G.v21)                               # G11^{-t} V21
    # (1,2) = -G11^{-1} G12 S^{-1} = -(G11^{-1} U12)(S^{-t} V12)^t
    u12, v12 = compress(-AU, matvec_t(Si, G.v12), trunc)
    # (2,1) = -S^{-1} G21 G11^{-1} = -(S^{-1} U21)(G11^{-t} V21)^t
    u21, v21 = compress(-SiU, ATV, trunc)
    # (1,1) = G11^{-1} + (G11^{-1} U12)(V12^t S^{-1} U21)(G11^{-t} V21)^t
    a11 = add(A, lowrank_like(AU @ (G.v12.T @ SiU), ATV, A), trunc)
    return HM(G.n, a11=a11, a22=Si, u12=u12, v12=v12, u21=u21, v21=v21)


def diagmul_left(d, G):
    """hdiagmul(D, G) = D G for diagonal D = diag(d)."""
    if G.leaf:
        return HM(G.n, d=d[:, None] * G.d)
    n1 = G.n1
    return HM(G.n, a11=diagmul_left(d[:n1], G.a11), a22=diagmul_left(d[n1:], G.a22),
              u12=d[:n1, None] * G.u12, v12=G.v12, u21=d[n1:, None] * G.u21, v21=G.v21)


def diagmul_right(G, d):
    """hdiagmul(G, D) = G D for diagonal D = diag(d)."""
    if G.leaf:
        return HM(G.n, d=G.d * d[None, :])
    n1 = G.n1
    return HM(G.n, a11=diagmul_right(G.a11, d[:n1]), a22=diagmul_right(G.a22, d[n1:]),
              u12=G.u12, v12=d[n1:, None] * G.v12, u21=G.u21, v21=d[:n1, None] * G.v21)


def max_rank(G):
    if G.leaf:
        return 0
    return max(G.u12.shape[1], G.u21.shape[1], max_rank(G.a11), max_rank(G.a22))


def factor(st: assemble.Stencil, leaf, trunc):
    """Alg. 2.3: T~_1 = hinv(A_11); S~_m = hsub(A_mm, hdiagmul(A_{m,m-1},
    hdiagmul(T~_{m-1}, A_{m-1,m}))), T~_m = hinv(S~_m)."""
    n = st.n
    a = couplings(st)
    T = []
    for m in range(1, n + 1):
        d, up, _ = assemble.layer_blocks(st, m)
        lo = st.W[m - 1, 1:]
        Ah = tridiag(d.astype(complex), up.astype(complex), lo.astype(complex), leaf)
        if m == 1:
            S = Ah
        else:
            am = a[m - 2]
            S = add(Ah, diagmul_left(am, diagmul_right(T[-1], am)), trunc, alpha=-1.0)
        T.append(inv(S, trunc))
    return T


def solve(st: assemble.Stencil, T, f):
    """Alg. 2.4: the sweep with hmatvec(T~_m, .) -- the preconditioner M."""
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
