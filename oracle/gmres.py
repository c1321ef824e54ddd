"""GMRES in FP64 (Sec. 2.4: the preconditioned system is solved by GMRES).

Two textbook variants (Saad, Iterative Methods for Sparse Linear Systems):

* `fgmres`: right-preconditioned flexible GMRES (Saad Alg. 9.6).  It
  minimizes the true residual ||f - A u||_2 over the span of the
  preconditioned Arnoldi vectors, so the monitored residual is the one the
  stopping rule is stated in.
* `left_gmres`: GMRES on M A u = M f, the paper's form, with the residual
  of the preconditioned system monitored.

Both start from x0 = 0 unless given, use modified Gram-Schmidt and Givens
rotations, restart every `restart` steps and stop when the relative
residual (true residual for fgmres) is <= tol.
"""
import numpy as np


def _givens(a, b):
    """Complex Givens rotation (c real, s complex) zeroing b in (a, b)."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def fgmres(apply_A, f, precond=None, tol=1e-6, restart=50, maxit=200, x0=None):
    """Returns (x, iterations, true relative residual history per restart)."""
    f = np.asarray(f, dtype=np.complex128)
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.complex128)
    fnorm = np.linalg.norm(f)
    if fnorm == 0:
        return np.zeros_like(f), 0, [0.0]
    history = []
    its = 0
    r = f - apply_A(x)
    beta = np.linalg.norm(r)
    history.append(beta / fnorm)
    while beta / fnorm > tol and its < maxit:
        m = min(restart, maxit - its)
        V = np.zeros((m + 1, f.size), dtype=np.complex128)
        Z = np.zeros((m, f.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for k in range(m):
            Z[k] = M(V[k])
            w = apply_A(Z[k])
            for i in range(k + 1):
                H[i, k] = np.vdot(V[i], w)
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -np.conj(sn[i]) * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            cs[k], sn[k] = _givens(H[k, k], H[k + 1, k])
            H[k, k] = cs[k] * H[k, k] + sn[k] * H[k + 1, k]
            H[k + 1, k] = 0.0
            g[k + 1] = -np.conj(sn[k]) * g[k]
            g[k] = cs[k] * g[k]
            its += 1
            if abs(g[k + 1]) / fnorm <= tol:
                break
        kk = k + 1
        y = np.linalg.solve(np.triu(H[:kk, :kk]), g[:kk])
        x = x + y @ Z[:kk]
        r = f - apply_A(x)
        beta = np.linalg.norm(r)
        history.append(beta / fnorm)
    return x, its, history


def left_gmres(apply_A, f, precond, tol=1e-3, restart=50, maxit=200):
    """GMRES on M A u = M f (the paper's left-preconditioned form).

    Returns (x, iterations, preconditioned relative residual)."""
    MA = lambda v: precond(apply_A(v))
    Mf = precond(np.asarray(f, dtype=np.complex128))
    x, its, hist = fgmres(MA, Mf, precond=None, tol=tol, restart=restart, maxit=maxit)
    return x, its, hist[-1]
