"""Pins of the oracle's 3D method (CPU only): the 7-point PML operator, the
exact face-by-face sweep and the strongly admissible face H-matrices."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gmres, hmatrix, strong, threed as T3

SIDES = (1, 2, 2, 1, 1, 2)


def _medium(n, seed):
    return 1 + 0.3 * np.random.default_rng(seed).random((n, n, n))


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _gauss(n, centre, width_in_h=1.5):
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    s = width_in_h * h
    r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2
    return np.exp(-r2 / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5, np.sqrt(r2), s


# ---------------------------------------------------------------- the operator

def test_operator_is_symmetric_with_closed_form_row_sums():
    n, om = 7, 2 * np.pi * 1.5
    c = _medium(n, 1)
    st = T3.stencil(c, om, SIDES)
    A = T3.matrix(st)
    assert abs(A - A.T).max() == 0
    assert A.nnz == 7 * n ** 3 - 6 * n * n            # 7-point stencil, zero boundary
    rs = np.asarray(A.sum(axis=1)).reshape(n, n, n)
    ref = om ** 2 / (st.s123 * c ** 2)
    inner = (slice(1, -1),) * 3
    np.testing.assert_allclose(rs[inner], ref[inner], rtol=1e-13)
    u = _rand(np.random.default_rng(2), 2, n ** 3)
    np.testing.assert_allclose(T3.apply(st, u), (A @ u.T).T, rtol=0, atol=1e-10 * abs(A).max())


@pytest.mark.parametrize("n", [7, 9])
def test_separable_closed_form_matches_sparse_lu(n):
    om = 2 * np.pi * 1.5
    st = T3.stencil(np.ones((n, n, n)), om, SIDES)
    f = _rand(np.random.default_rng(n), n ** 3)
    ue = spla.spsolve(T3.matrix(st).tocsc(), f)
    np.testing.assert_allclose(T3.solve_constant(n, om, SIDES, 1.0, f), ue, rtol=0, atol=1e-11 * abs(ue).max())


def test_point_source_converges_to_the_free_space_green_function():
    # c = 1, layers of a quarter of the side, a Gaussian of unit mass at the
    # centre: outside its support the field is -exp(-k^2 s^2 / 2) e^{ikr}/(4 pi r)
    om = 2 * np.pi * 4
    errs = []
    for n in (31, 63, 127):
        f, r, s = _gauss(n, (0.5, 0.5, 0.5))
        u = T3.solve_constant(n, om, (n + 1) // 4, 1.0, f.ravel()).reshape(n, n, n)
        ref = -np.exp(-(om * s) ** 2 / 2) * np.exp(1j * om * r) / (4 * np.pi * np.maximum(r, 1e-12))
        shell = (r >= 0.1) & (r <= 0.2)
        errs.append(np.linalg.norm(u[shell] - ref[shell]) / np.linalg.norm(ref[shell]))
        if n == 31:   # the incoming convention (complex conjugate) is far off
            assert np.linalg.norm(u[shell] - np.conj(ref[shell])) / np.linalg.norm(ref[shell]) > 0.5
    assert errs[0] / errs[1] >= 3.5 and errs[1] / errs[2] >= 3.5
    assert errs[2] <= 1e-2


def test_dropped_face_coupling_is_caught_by_the_closed_form():
    # Planted mistake: the x3 couplings below each point left out.
    n, om = 7, 2 * np.pi * 1.5
    st = T3.stencil(np.ones((n, n, n)), om, SIDES)
    st.Z0 = np.zeros_like(st.Z0)
    f = _rand(np.random.default_rng(3), n ** 3)
    bad = spla.spsolve(T3.matrix(st).tocsc(), f)
    good = T3.solve_constant(n, om, SIDES, 1.0, f)
    assert np.abs(bad - good).max() > 1e-3 * np.abs(good).max()


# ---------------------------------------------------------------- exact sweep

@pytest.mark.parametrize("n", [7, 9])
def test_exact_face_sweep_is_the_inverse(n):
    st = T3.stencil(_medium(n, n), 2 * np.pi * 1.5, SIDES)
    f = _rand(np.random.default_rng(5), 2, n ** 3)
    ue = spla.spsolve(T3.matrix(st).tocsc(), f.T).T
    u = T3.solve_exact(st, T3.factor_exact(st), f)
    np.testing.assert_allclose(u, ue, rtol=0, atol=1e-11 * abs(ue).max())


def test_face_schur_inverse_is_the_half_space_green_function():
    n = 5
    st = T3.stencil(_medium(n, 7), 2 * np.pi, SIDES)
    T = T3.factor_exact(st)
    A = T3.matrix(st).toarray()
    N2 = n * n
    for m in (1, 3):
        sub = A[:(m + 1) * N2, :(m + 1) * N2]
        np.testing.assert_allclose(T[m], np.linalg.inv(sub)[m * N2:, m * N2:], rtol=0, atol=1e-12 * abs(T[m]).max())


# ---------------------------------------------------------------- face H-matrices

def _segment_starts(n, levels):
    """Left ends of the 2^levels intervals of [0, n) cut by repeated bisection."""
    segs = [(0, n)]
    for _ in range(levels):
        segs = [p for lo, hi in segs for p in ((lo, lo + (hi - lo) // 2), (lo + (hi - lo) // 2, hi))]
    return [lo for lo, _ in segs]


@pytest.mark.parametrize("n, leaf", [(7, 4), (11, 9), (16, 16)])
def test_face_blocks_follow_the_quadtree_and_strong_admissibility(n, leaf):
    geo = T3.Face(n, leaf)
    assert sorted(geo.perm) == list(range(n * n))
    like = strong.zeros(n * n, leaf, geo)
    cover = np.zeros((n * n, n * n), int)

    def boxes(rng_):
        pts = geo.perm[rng_[0]:rng_[1]]
        i, j = pts % n, pts // n
        return i.min(), i.max() + 1, j.min(), j.max() + 1, len(pts)
    for b in strong.blocks(like):
        cover[b.t[0]:b.t[1], b.s[0]:b.s[1]] += 1
        for r in (b.t, b.s):                      # every cluster is a full box of points
            i0, i1, j0, j1, cnt = boxes(r)
            assert cnt == (i1 - i0) * (j1 - j0)
        if b.kind == "F":
            assert b.level % 2 == 0
            lq = b.level // 2
            starts = _segment_starts(n, lq)
            ti, tj = starts.index(boxes(b.t)[0]), starts.index(boxes(b.t)[2])
            si, sj = starts.index(boxes(b.s)[0]), starts.index(boxes(b.s)[2])
            assert max(abs(ti - si), abs(tj - sj)) > 1            # well separated
            assert max(abs(ti // 2 - si // 2), abs(tj // 2 - sj // 2)) <= 1   # parents are not
        else:
            assert b.kind == "D" and b.level == geo.L
            assert max(b.m, b.q) <= leaf
    np.testing.assert_array_equal(cover, 1)


def test_face_hmatrix_factorization_without_truncation_equals_the_dense_schur_factors():
    n = 7
    st = T3.stencil(_medium(n, 11), 2 * np.pi * 1.5, SIDES)
    Ts, geo = T3.factor_strong(st, 4, hmatrix.Trunc(), np.random.default_rng(0))
    P = geo.perm
    for t, tx in zip(Ts, T3.factor_exact(st)):
        np.testing.assert_allclose(strong.to_dense(t), tx[np.ix_(P, P)], rtol=0, atol=1e-12 * abs(tx).max())
    f = _rand(np.random.default_rng(1), n ** 3)
    ue = spla.spsolve(T3.matrix(st).tocsc(), f)
    np.testing.assert_allclose(T3.solve_strong(st, Ts, geo, f), ue, rtol=0, atol=1e-11 * abs(ue).max())


def test_rank_two_face_hmatrices_precondition_gmres_to_the_solution():
    n = 15
    st = T3.stencil(_medium(n, 13), 2 * np.pi * 2, 3)
    f, _, _ = _gauss(n, (0.5, 0.5, 0.5))
    f = f.ravel().astype(complex)
    Ts, geo = T3.factor_strong(st, 16, hmatrix.Trunc(1e-6, 2), np.random.default_rng(3))
    assert max(strong.max_rank(t) for t in Ts) == 2
    u, its, _ = gmres.fgmres(lambda v: T3.apply(st, v), f, precond=lambda v: T3.solve_strong(st, Ts, geo, v),
                             tol=1e-10)
    ue = spla.spsolve(T3.matrix(st).tocsc(), f)
    assert np.abs(u - ue).max() <= 1e-8 * np.abs(ue).max()
    assert its <= 10
