"""Exact sweeping factorization and solve (Sec. 2.1, Algs. 2.1 and 2.2).

Factorization (block LDL^t, eq. Afact): with T_m = S_m^{-1},

  S_1 = A_{1,1},   S_m = A_{m,m} - A_{m,m-1} T_{m-1} A_{m-1,m}   (m = 2..n).

A_{m,m-1} = A_{m-1,m}^t is diagonal, so the update is a diagonal scaling
of T_{m-1} on both sides.  The solve runs the forward substitution
(u_{m+1} -= A_{m+1,m} T_m u_m), the block-diagonal solve (u_m = T_m u_m)
and the backward substitution (u_m -= T_m A_{m,m+1} u_{m+1}).  The
products T_m u_m of the forward loop and of the diagonal loop are the
same, so they are computed once.

Every T_m is kept dense (n x n): O(n^4) work and O(n^3) storage, which is
why the paper replaces them by H-matrices.  Here it is the exact version
of the method, used as the reference preconditioner.
"""
import numpy as np

from . import assemble


def couplings(st: assemble.Stencil):
    """a[m] = diagonal of A_{m+1,m} (1-based m = 1..n-1), shape (n-1, n)."""
    return st.S[1:].copy()


def factor(st: assemble.Stencil):
    """Dense T_1..T_n (list of n x n complex128)."""
    n = st.n
    a = couplings(st)
    T = []
    for m in range(1, n + 1):
        S = assemble.layer_tridiag(st, m).astype(np.complex128)
        if m > 1:
            am = a[m - 2]
            S = S - am[:, None] * T[-1] * am[None, :]
        T.append(np.linalg.inv(S))
    return T


def solve(st: assemble.Stencil, T, f):
    """u = M f with the factors T (Alg. 2.2); exact inverse when T is exact."""
    n = st.n
    a = couplings(st)
    f = np.asarray(f, dtype=np.complex128)
    single = f.ndim == 1
    F = f.reshape(-1, n, n)
    U = np.empty_like(F)
    for k in range(F.shape[0]):
        u = F[k].copy()
        w = np.empty_like(u)
        # forward substitution; w_m = T_m u_m is reused by the diagonal solve
        for m in range(n):
            if m > 0:
                u[m] = u[m] - a[m - 1] * w[m - 1]
            w[m] = T[m] @ u[m]
        # backward substitution
        u[n - 1] = w[n - 1]
        for m in range(n - 2, -1, -1):
            u[m] = w[m] - T[m] @ (a[m] * u[m + 1])
        U[k] = u
    U = U.reshape(-1, n * n)
    return U[0] if single else U


def leading_inverse_block(st: assemble.Stencil, m):
    """[(A restricted to layers 1..m)^{-1}]_{m,m}: the discrete half-space
    Green's function on row m with zero data on row m+1 (Sec. 2.2)."""
    n = st.n
    A = assemble.matrix(st).toarray()
    k = m * n
    Ginv = np.linalg.inv(A[:k, :k])
    return Ginv[k - n:, k - n:]


def solve_direction(st: assemble.Stencil, f, direction, T=None):
    """The exact sweep of Algs. 2.1/2.2 in one of the four directions
    (Sec. 2.4): relabel the grid so that the layers run along the chosen
    direction, sweep there, and map the result back.  T: the frame's
    factors if already computed.  Returns (u, T)."""
    n = st.n
    sp = assemble.permuted(st, direction)
    if T is None:
        T = factor(sp)
    F = np.asarray(f, dtype=np.complex128).reshape(-1, n, n)
    Ff = np.ascontiguousarray(assemble.to_frame(F, direction)).reshape(-1, n * n)
    Uf = solve(sp, T, Ff).reshape(-1, n, n)
    U = np.ascontiguousarray(assemble.from_frame(Uf, direction)).reshape(-1, n * n)
    return (U[0] if np.asarray(f).ndim == 1 else U), T
