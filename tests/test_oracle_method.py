"""Pins of the oracle's sweeping factorization, H-matrix algebra, GMRES and
adjoint gradient (CPU only)."""
import numpy as np
import pytest

from oracle import assemble, direct, gmres, gradient, hmatrix, sweep
import workloads as W


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------- exact sweep

@pytest.mark.parametrize("n", [7, 15])
def test_schur_inverse_is_half_space_green_function(n):
    # Sec. 2.2: T_m is the (m, m) block of the inverse of A restricted to layers 1..m.
    st = assemble.stencil(W.random_field_medium(n, 5), 2 * np.pi * 2, 2)
    T = sweep.factor(st)
    for m in range(1, n + 1):
        G = sweep.leading_inverse_block(st, m)
        assert _rel(T[m - 1], G) < 1e-12


def test_schur_inverses_are_symmetric():
    n = 31
    st = assemble.stencil(W.random_field_medium(n, 5), 2 * np.pi * 4, 5)
    for Tm in sweep.factor(st):
        assert np.linalg.norm(Tm - Tm.T) / np.linalg.norm(Tm) < 1e-12


def test_exact_sweep_is_the_inverse_and_gmres_takes_one_iteration():
    # helm63 workload: n = 63, omega = 2 pi 8, c = 1, PML 12, centre source.
    wl = W.get("helm63_dense_c1")
    st = assemble.stencil(wl.velocity(), wl.omega, wl.pml)
    f = wl.sources()[0]
    T = sweep.factor(st)
    u_lu = direct.solve_sparse(st, f)
    u_sw = sweep.solve(st, T, f)
    assert _rel(u_sw, u_lu) < 1e-11
    x, its, hist = gmres.fgmres(lambda v: assemble.apply(st, v), f,
                                precond=lambda v: sweep.solve(st, T, v), tol=1e-12)
    assert its == 1
    assert hist[-1] <= 1e-12


def test_sweep_with_perturbed_factor_is_not_exact():
    # Planted mistake: dropping the coupling term of the Schur update.
    n = 15
    st = assemble.stencil(W.random_field_medium(n, 5), 2 * np.pi * 2, 3)
    T_bad = [np.linalg.inv(assemble.layer_tridiag(st, m)) for m in range(1, n + 1)]
    f = W.gaussian_source(n, (0.5, 0.5)).ravel()
    assert _rel(sweep.solve(st, T_bad, f), direct.solve_sparse(st, f)) > 1e-2


# ---------------------------------------------------------------- GMRES

def test_fgmres_textbook_properties():
    rng = np.random.default_rng(1)
    k = 30
    A = np.eye(k) * 4 + rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
    b = rng.standard_normal(k) + 1j * rng.standard_normal(k)
    x, its, hist = gmres.fgmres(lambda v: A @ v, b, tol=1e-13, restart=k)
    assert its <= k
    assert _rel(x, np.linalg.solve(A, b)) < 1e-11
    # restarted GMRES converges to the same solution when the spectrum is
    # well separated from the origin (GMRES(m) may stagnate otherwise)
    A2 = A + 8 * np.eye(k)
    x2, its2, _ = gmres.fgmres(lambda v: A2 @ v, b, tol=1e-12, restart=7, maxit=500)
    assert _rel(x2, np.linalg.solve(A2, b)) < 1e-10
    # exact preconditioner: one iteration (right and left forms)
    Ainv = np.linalg.inv(A)
    _, its3, _ = gmres.fgmres(lambda v: A @ v, b, precond=lambda v: Ainv @ v, tol=1e-12)
    assert its3 == 1
    _, its4, _ = gmres.left_gmres(lambda v: A @ v, b, lambda v: Ainv @ v, tol=1e-12)
    assert its4 == 1


def test_fgmres_residual_estimate_matches_true_residual():
    rng = np.random.default_rng(2)
    k = 40
    A = np.diag(np.linspace(1, 10, k)) + 0.3 * rng.standard_normal((k, k))
    b = rng.standard_normal(k).astype(complex)
    x, its, hist = gmres.fgmres(lambda v: A @ v, b, tol=1e-8, restart=60)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) == pytest.approx(hist[-1], rel=1e-6)
    assert hist[-1] <= 1e-8


# ---------------------------------------------------------------- H-matrix algebra

def _random_hm(n, leaf, rank, rng, sym=False):
    if n <= leaf:
        d = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 3 * n * np.eye(n)
        return hmatrix.HM(n, d=(d + d.T) / 2 if sym else d)
    n1 = n // 2
    cplx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    u12, v12 = cplx(n1, rank), cplx(n - n1, rank)
    if sym:
        u21, v21 = v12.copy(), u12.copy()
    else:
        u21, v21 = cplx(n - n1, rank), cplx(n1, rank)
    return hmatrix.HM(n, a11=_random_hm(n1, leaf, rank, rng, sym), a22=_random_hm(n - n1, leaf, rank, rng, sym),
                      u12=u12, v12=v12, u21=u21, v21=v21)


@pytest.mark.parametrize("n,leaf", [(64, 8), (45, 6)])
def test_hmatrix_operations_exact_without_truncation(n, leaf):
    rng = np.random.default_rng(3)
    G = _random_hm(n, leaf, 2, rng)
    H = _random_hm(n, leaf, 3, rng)
    Gd, Hd = hmatrix.to_dense(G), hmatrix.to_dense(H)
    exact = hmatrix.Trunc()
    X = rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))
    assert _rel(hmatrix.matvec(G, X), Gd @ X) < 1e-13
    assert _rel(hmatrix.matvec_t(G, X), Gd.T @ X) < 1e-13
    assert _rel(hmatrix.to_dense(hmatrix.add(G, H, exact)), Gd + Hd) < 1e-13
    assert _rel(hmatrix.to_dense(hmatrix.add(G, H, exact, -1.0)), Gd - Hd) < 1e-13
    assert _rel(hmatrix.to_dense(hmatrix.mul(G, H, exact)), Gd @ Hd) < 1e-12
    assert _rel(hmatrix.to_dense(hmatrix.inv(G, exact)), np.linalg.inv(Gd)) < 1e-11
    d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert _rel(hmatrix.to_dense(hmatrix.diagmul_left(d, G)), d[:, None] * Gd) < 1e-14
    assert _rel(hmatrix.to_dense(hmatrix.diagmul_right(G, d)), Gd * d[None, :]) < 1e-14
    P = rng.standard_normal((n, 2)) + 0j
    assert _rel(hmatrix.to_dense(hmatrix.lowrank_like(P, P, G)), P @ P.T) < 1e-14


def test_compress_truncation_error_bound():
    # Eckart-Young: the rank-k truncation error in the 2-norm is sigma_{k+1}.
    rng = np.random.default_rng(4)
    U = rng.standard_normal((50, 12)) @ np.diag(10.0 ** -np.arange(12))
    V = rng.standard_normal((40, 12)) + 1j * rng.standard_normal((40, 12))
    M = U @ V.T
    s = np.linalg.svd(M, compute_uv=False)
    for tol, rmax in [(1e-6, None), (1e-3, None), (0.0, 4), (1e-9, 6)]:
        u, v = hmatrix.compress(U, V, hmatrix.Trunc(tol, rmax))
        k = u.shape[1]
        expect_k = int(np.sum(s > tol * s[0])) if tol > 0 else 12
        if rmax is not None:
            expect_k = min(expect_k, rmax)
        assert k == expect_k
        err = np.linalg.norm(M - u @ v.T, 2)
        assert err <= s[k] * (1 + 1e-6) + 1e-12 * s[0]


def test_hmatrix_factorization_without_truncation_equals_dense_schur():
    n = 31
    st = assemble.stencil(W.random_field_medium(n, 9), 2 * np.pi * 3, 5)
    T = sweep.factor(st)
    Th = hmatrix.factor(st, 4, hmatrix.Trunc())
    for Td, Tm in zip(T, Th):
        assert _rel(hmatrix.to_dense(Tm), Td) < 1e-10


def test_hmatrix_sweep_without_truncation_is_the_exact_inverse():
    # Alg. 2.4 with untruncated H-factors is Alg. 2.2 with the dense factors,
    # and both give u = A^{-1} f (ragged bisection at n = 27 included).
    for n, leaf in ((15, 4), (27, 4)):
        st = assemble.stencil(W.random_field_medium(n, 13), 2 * np.pi * 2.5, 3)
        T = sweep.factor(st)
        Th = hmatrix.factor(st, leaf, hmatrix.Trunc())
        rng = np.random.default_rng(n)
        f = rng.standard_normal((2, n * n)) + 1j * rng.standard_normal((2, n * n))
        uh = hmatrix.solve(st, Th, f)
        assert _rel(uh, sweep.solve(st, T, f)) < 1e-11
        assert _rel(uh, direct.solve_dense(st, f)) < 1e-10
    # planted mistake: dropping the backward substitution is caught
    n = 15
    st = assemble.stencil(W.random_field_medium(n, 13), 2 * np.pi * 2.5, 3)
    Th = hmatrix.factor(st, 4, hmatrix.Trunc())
    f = W.gaussian_source(n, (0.5, 0.5)).ravel()
    a = sweep.couplings(st)
    F = f.reshape(n, n).copy()
    w = np.empty_like(F)
    for m in range(n):
        if m > 0:
            F[m] -= a[m - 1] * w[m - 1]
        w[m] = hmatrix.matvec(Th[m], F[m])
    assert _rel(w.ravel(), direct.solve_dense(st, f)) > 1e-3


def test_compressed_sweep_preconditions_gmres():
    # Truncated factors (rank <= 8, tol 1e-6) still precondition well and GMRES
    # reaches the exact solution.
    n = 63
    st = assemble.stencil(W.random_field_medium(n, 9), 2 * np.pi * 8, 8)
    Th = hmatrix.factor(st, 8, hmatrix.Trunc(1e-6, 8))
    assert max(hmatrix.max_rank(t) for t in Th) <= 8
    f = W.gaussian_source(n, (0.5, 0.5)).ravel()
    x, its, hist = gmres.fgmres(lambda v: assemble.apply(st, v), f,
                                precond=lambda v: hmatrix.solve(st, Th, v), tol=1e-10)
    assert hist[-1] <= 1e-10
    assert its <= 6
    assert _rel(x, direct.solve_sparse(st, f)) < 1e-8


# ---------------------------------------------------------------- gradient

def test_adjoint_gradient_matches_central_differences():
    n, npml = 31, 4
    omega = 2 * np.pi * 4
    c_true = W.random_field_medium(n, 5)
    c0 = W.constant_medium(n)
    F = np.stack([W.gaussian_source(n, p).ravel() for p in W.bottom_row_sources(n, npml, 4, margin=3)])
    rec = W.top_row_receivers(n, npml, 16, margin=3)
    _, _, U_true = gradient.forward(c_true, omega, npml, F)
    data = U_true[:, rec]
    J, g = gradient.adjoint_gradient(c0, omega, npml, F, rec, data)
    assert J > 0
    rng = np.random.default_rng(6)
    eps = 2e-3 / omega
    for _ in range(4):
        v = W.random_field_medium(n, int(rng.integers(1 << 30)), amplitude=1.0) - 1.0
        fd = gradient.central_difference(c0, omega, npml, F, rec, data, v, eps)
        ad = float(np.sum(g * v))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-12


def test_source_gradient_matches_central_differences():
    # dJ/dRe f + i dJ/dIm f = conj(mu): checked along random complex source
    # perturbations, whose directional derivative is Re sum conj(grad_f) v.
    n, npml = 15, 3
    omega = 2 * np.pi * 2
    c0 = W.random_field_medium(n, 21)
    F = np.stack([W.gaussian_source(n, p).ravel() for p in ((0.4, 0.3), (0.6, 0.35))])
    rec = W.top_row_receivers(n, npml, 5, margin=1)
    data = np.full((2, rec.size), 0.02 + 0.01j)
    J, _, _, Mu = gradient.adjoint_state(c0, omega, npml, F, rec, data)
    grad_f = np.conj(Mu)
    rng = np.random.default_rng(8)
    eps = 1e-4
    for _ in range(3):
        v = rng.standard_normal(F.shape) + 1j * rng.standard_normal(F.shape)
        jp = gradient.misfit(c0, omega, npml, F + eps * v, rec, data)
        jm = gradient.misfit(c0, omega, npml, F - eps * v, rec, data)
        fd = (jp - jm) / (2 * eps)
        ad = float(np.real(np.sum(np.conj(grad_f) * v)))
        assert abs(fd - ad) <= 1e-7 * abs(ad)
    # planted mistake: the adjoint field itself (no conjugate) is not the gradient
    v = rng.standard_normal(F.shape) + 1j * rng.standard_normal(F.shape)
    fd = (gradient.misfit(c0, omega, npml, F + eps * v, rec, data)
          - gradient.misfit(c0, omega, npml, F - eps * v, rec, data)) / (2 * eps)
    assert abs(float(np.real(np.sum(np.conj(Mu) * v))) - fd) > 1e-3 * abs(fd)


def test_wrong_adjoint_sign_is_caught_by_differences():
    # Planted mistake: the conjugate of the adjoint field gives a wrong gradient.
    n, npml = 15, 3
    omega = 2 * np.pi * 2
    c0 = W.constant_medium(n)
    F = W.gaussian_source(n, (0.5, 0.3)).reshape(1, -1)
    rec = W.top_row_receivers(n, npml, 5, margin=1)
    data = np.ones((1, rec.size), complex) * 0.01
    st, lu, U = gradient.forward(c0, omega, npml, F)
    r = U[:, rec] - data
    G = np.zeros_like(U)
    G[:, rec] = r
    Mu_bad = lu.solve(G)              # missing conj
    dD = 2 * omega ** 2 / (st.s1s2 * st.c ** 3)
    g_bad = np.real(Mu_bad.reshape(-1, n, n) * U.reshape(-1, n, n) * dD[None]).sum(0)
    _, g = gradient.adjoint_gradient(c0, omega, npml, F, rec, data)
    v = W.random_field_medium(n, 77, amplitude=1.0) - 1.0
    fd = gradient.central_difference(c0, omega, npml, F, rec, data, v, 1e-4 / omega)
    assert abs(np.sum(g * v) - fd) < 1e-6 * abs(fd)
    assert abs(np.sum(g_bad * v) - fd) > 1e-2 * abs(fd)


# ---------------------------------------------------------------- inputs

def test_workload_inputs_are_seeded_and_in_range():
    a = W.random_field_medium(63, 1)
    b = W.random_field_medium(63, 1)
    np.testing.assert_array_equal(a, b)
    assert a.min() >= 0.7 - 1e-12 and a.max() <= 1.3 + 1e-12
    assert np.max(np.abs(a - 1)) == pytest.approx(0.3)
    f = W.gaussian_source(255, (0.5, 0.5))
    h = 1 / 256
    assert np.sum(f.real) * h * h == pytest.approx(1.0, rel=1e-6)
    lens = W.lens_medium(63)
    assert lens.min() >= 0.6 and lens.max() <= 1.0
