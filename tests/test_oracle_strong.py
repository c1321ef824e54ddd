"""Pins of the oracle's strongly admissible H-matrices, randomized SVD and
the sweeping factorization in that format (CPU only)."""
import numpy as np
import pytest

from oracle import assemble, direct, gmres, hmatrix, strong, sweep
import workloads as W

EXACT = hmatrix.Trunc()


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _unitary(rng, n):
    q, r = np.linalg.qr(_rand(rng, n, n))
    return q * (np.diag(r) / np.abs(np.diag(r)))


# ---------------------------------------------------------------- the format

@pytest.mark.parametrize("n, leaf", [(32, 4), (37, 4), (63, 8), (100, 6)])
def test_blocks_tile_the_matrix_and_follow_strong_admissibility(n, leaf):
    L = strong.depth(n, leaf)
    like = strong.zeros(n, leaf)
    cover = np.zeros((n, n), int)
    for b in strong.blocks(like):
        cover[b.t[0]:b.t[1], b.s[0]:b.s[1]] += 1
        # position of each cluster within its level, from the bisection itself
        pos = []
        for c in (b.t, b.s):
            lo, hi, k = 0, n, 0
            for _ in range(b.level):
                mid = lo + (hi - lo) // 2
                k = 2 * k + (c[0] >= mid)
                lo, hi = (mid, hi) if c[0] >= mid else (lo, mid)
            assert (lo, hi) == c
            pos.append(k)
        gap = abs(pos[0] - pos[1])
        if b.kind == "F":
            assert gap >= 2                              # a cluster lies between them
            assert abs(pos[0] // 2 - pos[1] // 2) <= 1   # parents not well separated
        else:
            assert gap <= 1 and b.kind == "D" and b.level == L
        assert max(b.m, b.q) <= leaf or b.kind == "F"
    np.testing.assert_array_equal(cover, 1)


def test_well_separated_is_distance_at_least_width():
    assert not strong.well_separated((0, 4), (4, 8))        # adjacent: distance 1
    assert strong.well_separated((0, 4), (8, 12))           # distance 5 >= 4
    assert not strong.well_separated((0, 4), (0, 4))
    assert strong.well_separated((0, 3), (6, 10))           # distance 4 >= 4
    assert not strong.well_separated((0, 3), (6, 11))       # distance 4 < 5


# ---------------------------------------------------------------- exact H-arithmetic

@pytest.mark.parametrize("n, leaf", [(37, 4), (64, 8)])
def test_operations_without_truncation_equal_dense_algebra(n, leaf):
    rng = np.random.default_rng(11)
    like = strong.zeros(n, leaf)
    M = _rand(rng, n, n) + 8 * np.eye(n)
    N = _rand(rng, n, n)
    A = strong.from_dense(M, like, EXACT)
    B = strong.from_dense(N, like, EXACT)
    X = _rand(rng, n, 3)
    np.testing.assert_allclose(strong.to_dense(A), M, atol=1e-12)
    np.testing.assert_allclose(strong.matvec(A, X), M @ X, atol=1e-11)
    np.testing.assert_allclose(strong.matvec_t(A, X), M.T @ X, atol=1e-11)
    np.testing.assert_allclose(strong.to_dense(strong.add(A, B, EXACT, -1.0)), M - N, atol=1e-11)
    P = strong.mul(A, B, like, EXACT, rng)
    assert np.abs(strong.to_dense(P) - M @ N).max() <= 1e-12 * np.abs(M @ N).max()
    I = strong.inv(A, EXACT, rng)
    assert np.abs(strong.to_dense(I) @ M - np.eye(n)).max() <= 1e-11
    d = _rand(rng, n)
    np.testing.assert_allclose(strong.to_dense(strong.diagmul_left(d, A)), d[:, None] * M, atol=1e-11)
    np.testing.assert_allclose(strong.to_dense(strong.diagmul_right(A, d)), M * d[None, :], atol=1e-11)


def test_truncated_blocks_obey_the_rank_cap_and_eckart_young():
    rng = np.random.default_rng(3)
    n, leaf, R = 64, 8, 2
    like = strong.zeros(n, leaf)
    M = _rand(rng, n, n)
    A = strong.from_dense(M, like, hmatrix.Trunc(0.0, R))
    assert strong.max_rank(A) == R
    for b in strong.blocks(A):
        if b.kind == "F":
            s = np.linalg.svd(M[b.t[0]:b.t[1], b.s[0]:b.s[1]], compute_uv=False)
            err = np.linalg.norm(M[b.t[0]:b.t[1], b.s[0]:b.s[1]] - b.u @ b.v.T, 2)
            assert err == pytest.approx(s[R], rel=1e-10)


# ---------------------------------------------------------------- randomized SVD

def _operator(rng, m, q, sv):
    U, V = _unitary(rng, m)[:, :len(sv)], _unitary(rng, q)[:, :len(sv)]
    return (U * sv) @ V.conj().T


@pytest.mark.parametrize("rank", [1, 2, 5])
def test_randomized_svd_is_exact_for_low_rank_operators(rank):
    rng = np.random.default_rng(rank)
    A = _operator(rng, 40, 30, np.linspace(3.0, 1.0, rank))
    U, V = strong.rsvd(lambda X: A @ X, lambda Y: A.T @ Y, 40, 30, hmatrix.Trunc(1e-12, 5), rng)
    assert U.shape[1] == rank
    assert np.abs(U @ V.T - A).max() <= 1e-13


def test_randomized_svd_error_lies_within_the_probabilistic_bound():
    # Halko-Martinsson-Tropp (2011), Sec. 1.5: with k + p Gaussian samples,
    # ||A - Q Q^* A|| <= (1 + 11 sqrt(k + p) sqrt(min(m, n))) sigma_{k+1}
    # except with probability at most 6 p^-p; the rank-k result can be no
    # better than sigma_{k+1} (Eckart-Young) and its truncation adds at most
    # sigma_{k+1} more.
    m, q, k, p = 60, 50, 2, strong.OVERSAMPLE
    sv = 0.5 ** np.arange(min(m, q))
    bound = 1 + 11 * np.sqrt(k + p) * np.sqrt(min(m, q))
    for seed in range(10):
        rng = np.random.default_rng(100 + seed)
        A = _operator(rng, m, q, sv)
        U, V = strong.rsvd(lambda X: A @ X, lambda Y: A.T @ Y, m, q, hmatrix.Trunc(0.0, k), rng)
        err = np.linalg.norm(A - U @ V.T, 2)
        assert sv[k] * (1 - 1e-12) <= err <= (bound + 1) * sv[k]
        assert err <= 2.0 * sv[k]          # fast decay: close to the optimum in practice


def test_missing_conjugate_in_the_projection_is_caught(monkeypatch):
    # Planted mistake: B = Q^t (G H) instead of Q^H (G H).
    def bad(apply, apply_t, m, q, trunc, rng, oversample=strong.OVERSAMPLE):
        k = trunc.rmax if trunc.rmax is not None else min(m, q)
        ell = min(k + oversample, m, q)
        om = _rand(rng, q, ell)
        Q, _ = np.linalg.qr(apply(om))
        B = apply_t(Q).T
        W_, s, Zh = np.linalg.svd(B, full_matrices=False)
        r = trunc.keep(s)
        return Q @ (W_[:, :r] * s[:r]), Zh[:r].T
    rng = np.random.default_rng(7)
    n, leaf = 32, 4
    like = strong.zeros(n, leaf)
    M, N = _rand(rng, n, n), _rand(rng, n, n)
    A, B = strong.from_dense(M, like, EXACT), strong.from_dense(N, like, EXACT)
    monkeypatch.setattr(strong, "rsvd", bad)
    P = strong.mul(A, B, like, EXACT, rng)
    assert np.abs(strong.to_dense(P) - M @ N).max() > 1e-3 * np.abs(M @ N).max()


# ---------------------------------------------------------------- the factorization

def test_factorization_without_truncation_equals_the_dense_schur_factors():
    n = 31
    st = assemble.stencil(W.random_field_medium(n, 3), 2 * np.pi * 3, 4)
    rng = np.random.default_rng(0)
    T = strong.factor(st, 4, EXACT, rng)
    Td = sweep.factor(st)
    for t, td in zip(T, Td):
        assert np.abs(strong.to_dense(t) - td).max() <= 1e-11 * np.abs(td).max()
    f = _rand(rng, n * n)
    np.testing.assert_allclose(strong.solve(st, T, f), sweep.solve(st, Td, f), rtol=0,
                               atol=1e-10 * np.abs(sweep.solve(st, Td, f)).max())


def test_rank_two_strong_factors_precondition_gmres_to_the_solution():
    n = 63
    st = assemble.stencil(W.random_field_medium(n, 1), 2 * np.pi * 8, 12)
    f = W.gaussian_source(n, (0.5, 0.5)).ravel()
    T = strong.factor(st, 8, hmatrix.Trunc(1e-6, 2), np.random.default_rng(5))
    assert max(strong.max_rank(t) for t in T) == 2
    u, its, _ = gmres.fgmres(lambda v: assemble.apply(st, v), f, precond=lambda v: strong.solve(st, T, v),
                             tol=1e-10)
    ue = direct.solve_sparse(st, f)
    assert np.abs(u - ue).max() <= 1e-8 * np.abs(ue).max()
    # the paper's rank-2 setting: a handful of iterations, fewer than the
    # weakly admissible factors of the same rank need
    Tw = hmatrix.factor(st, 8, hmatrix.Trunc(1e-6, 2))
    _, its_w, _ = gmres.fgmres(lambda v: assemble.apply(st, v), f, precond=lambda v: hmatrix.solve(st, Tw, v),
                               tol=1e-10)
    assert its <= 5 and its < its_w
