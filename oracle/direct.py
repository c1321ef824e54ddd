"""u = A^{-1} f written out: direct solves of the 5-point PML system.

The solution of the discrete problem has a plain definition, the unique
u with A u = f (A is nonsingular because the PML damps every mode), and
every preconditioned Krylov iteration converges to it.  Three independent
direct routes are provided:

* sparse LU (SuperLU with COLAMD ordering), any n;
* banded LU (LAPACK gbsv through scipy.linalg.solve_banded), bandwidth n;
* dense LU (numpy.linalg.solve), tiny grids only.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import assemble


class SparseLU:
    """Factor once, solve many right-hand sides."""

    def __init__(self, st: assemble.Stencil):
        self.st = st
        self.lu = spla.splu(assemble.matrix(st).tocsc(), permc_spec="COLAMD")

    def solve(self, f):
        f = np.asarray(f, dtype=np.complex128)
        if f.ndim == 1:
            return self.lu.solve(f)
        return np.stack([self.lu.solve(fi) for fi in f], axis=0)


def solve_sparse(st, f):
    return SparseLU(st).solve(f)


def banded_form(st: assemble.Stencil):
    """LAPACK band storage ab[n + i - j, j] = A[i, j] with n sub/super diagonals."""
    n = st.n
    N = n * n
    A = assemble.matrix(st).tocoo()
    ab = np.zeros((2 * n + 1, N), dtype=np.complex128)
    ab[n + A.row - A.col, A.col] = A.data
    return ab


def solve_banded(st, f):
    n = st.n
    ab = banded_form(st)
    f = np.asarray(f, dtype=np.complex128)
    rhs = f.T if f.ndim == 2 else f
    u = sla.solve_banded((n, n), ab, rhs, overwrite_ab=True, check_finite=False)
    return u.T if f.ndim == 2 else u


def solve_dense(st, f):
    A = assemble.matrix(st).toarray()
    f = np.asarray(f, dtype=np.complex128)
    return np.linalg.solve(A, f.T).T if f.ndim == 2 else np.linalg.solve(A, f)


def relative_residual(st, u, f):
    """||f - A u||_2 / ||f||_2 per right-hand side, in FP64."""
    r = np.asarray(f) - assemble.apply(st, u)
    if r.ndim == 1:
        return np.linalg.norm(r) / np.linalg.norm(f)
    return np.linalg.norm(r, axis=1) / np.linalg.norm(f, axis=1)
