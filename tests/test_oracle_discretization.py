"""Pins of the oracle's discretization and direct solvers (CPU only).

Each test checks the oracle against something other than itself: exact
algebraic structure, closed-form spectra, an independently built separable
operator, the free-space Hankel field, or brute-force dense algebra.
"""
import numpy as np
import pytest

from oracle import assemble, direct, fastdiag, hankel, pml, sweep
import workloads as W


def _stencil(n, omega, npml, c=None, C=pml.DEFAULT_C):
    c = W.constant_medium(n) if c is None else c
    return assemble.stencil(c, omega, npml, C)


def test_sigma_profile_shape():
    # eq. sigma: zero inside [eta, 1-eta], quadratic growth to C/eta at the walls, mirror symmetric.
    eta, C = 0.25, 7.0
    t = np.linspace(0, 1, 101)
    s = pml.sigma(t, eta, C)
    assert np.all(s[(t >= eta) & (t <= 1 - eta)] == 0)
    assert s[0] == pytest.approx(C / eta)
    assert s[-1] == pytest.approx(C / eta)
    np.testing.assert_allclose(s, s[::-1], rtol=0, atol=1e-12)
    # quadratic: sigma(eta/2) = (C/eta) / 4
    assert pml.sigma(np.array([eta / 2]), eta, C)[0] == pytest.approx(C / eta / 4)
    # outgoing damping: Im(1/s) = sigma/omega > 0
    z = 1.0 / pml.stretch(t, 3.0, eta, C)
    np.testing.assert_allclose(z.imag, s / 3.0, rtol=1e-14)


def test_operator_symmetric_bitwise_and_layer_structure():
    n = 31
    st = _stencil(n, 2 * np.pi * 3, 5, W.random_field_medium(n, 7))
    A = assemble.matrix(st)
    assert abs(A - A.T).max() == 0.0
    Ad = A.toarray()
    for m in range(2, n + 1):
        blk = Ad[(m - 1) * n:m * n, (m - 2) * n:(m - 1) * n]     # A_{m,m-1}
        assert np.count_nonzero(blk - np.diag(np.diag(blk))) == 0
        np.testing.assert_array_equal(blk, Ad[(m - 2) * n:(m - 1) * n, (m - 1) * n:m * n].T)
        Amm = Ad[(m - 1) * n:m * n, (m - 1) * n:m * n]
        np.testing.assert_array_equal(Amm, assemble.layer_tridiag(st, m))
    # no coupling beyond adjacent layers
    assert np.count_nonzero(Ad[2 * n:3 * n, 0:n]) == 0


def test_row_sums_of_interior_rows():
    n = 15
    c = W.random_field_medium(n, 3)
    st = _stencil(n, 2 * np.pi * 2, 4, c)
    A = assemble.matrix(st).toarray()
    rs = A.sum(axis=1).reshape(n, n)
    expect = st.omega ** 2 / (st.s1s2 * c ** 2)
    np.testing.assert_allclose(rs[1:-1, 1:-1], expect[1:-1, 1:-1], rtol=1e-13)


def test_without_pml_spectrum_is_closed_form():
    # pml = 0, constant c: A = Dirichlet 5-point Laplacian + omega^2/c^2, whose
    # eigenvalues are omega^2/c^2 - (4/h^2)(sin^2(k1 pi h/2) + sin^2(k2 pi h/2)).
    n, c0, omega = 9, 1.3, 5.0
    st = _stencil(n, omega, 0, W.constant_medium(n, c0))
    ev = np.sort(np.linalg.eigvals(assemble.matrix(st).toarray()).real)
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1)
    mu = (4 / h ** 2) * np.sin(k * np.pi * h / 2) ** 2
    expect = np.sort((omega ** 2 / c0 ** 2 - (mu[:, None] + mu[None, :])).ravel())
    np.testing.assert_allclose(ev, expect, rtol=1e-12, atol=1e-9)


def test_apply_matches_matrix():
    n = 20
    st = _stencil(n, 2 * np.pi * 2, 4, W.random_field_medium(n, 2))
    rng = np.random.default_rng(0)
    u = rng.standard_normal((3, n * n)) + 1j * rng.standard_normal((3, n * n))
    A = assemble.matrix(st)
    np.testing.assert_allclose(assemble.apply(st, u), (A @ u.T).T, rtol=1e-14, atol=0)


@pytest.mark.parametrize("n", [3, 7, 15])
def test_direct_solvers_agree_on_tiny_grids(n):
    c = W.random_field_medium(n, 11) if n > 3 else np.array([[1.0, 1.1, 0.9], [1.2, 1.0, 0.8], [1.0, 0.95, 1.05]])
    st = _stencil(n, 2 * np.pi * 1.5, max(1, n // 5), c)
    rng = np.random.default_rng(n)
    f = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    u_dense = direct.solve_dense(st, f)
    for u in (direct.solve_sparse(st, f), direct.solve_banded(st, f)):
        assert np.linalg.norm(u - u_dense) / np.linalg.norm(u_dense) < 1e-12
    assert direct.relative_residual(st, u_dense, f) < 1e-12


@pytest.mark.parametrize("n,npml,freq", [(63, 12, 8), (255, 16, 32)])
def test_sparse_lu_matches_fast_diagonalization(n, npml, freq):
    omega = 2 * np.pi * freq
    st = _stencil(n, omega, npml)
    f = W.gaussian_source(n, (0.5, 0.5)).ravel()
    u_lu = direct.solve_sparse(st, f)
    u_fd = fastdiag.solve_constant(n, omega, npml, 1.0, f)
    assert np.linalg.norm(u_lu - u_fd) / np.linalg.norm(u_fd) < 1e-10


def test_hankel_field_second_order_convergence():
    # c = 1, omega = 2 pi 4, absorbing layer 0.2 wide, centre source; compare on
    # the annulus 0.1 <= r <= 0.3 (outside source and layer).
    omega = 2 * np.pi * 4
    errs = []
    for n in (63, 127, 255):
        h = 1.0 / (n + 1)
        npml = int(round(0.2 / h))
        st = _stencil(n, omega, npml)
        f = W.gaussian_source(n, (0.5, 0.5)).ravel()
        u = direct.solve_sparse(st, f).reshape(n, n)
        ur, r = hankel.gaussian_field(n, omega, (0.5, 0.5))
        mask = (r >= 0.1) & (r <= 0.3)
        errs.append(np.linalg.norm(u[mask] - ur[mask]) / np.linalg.norm(ur[mask]))
    assert errs[-1] < 2e-2
    for a, b in zip(errs[:-1], errs[1:]):
        assert 3.5 < a / b < 4.5, errs


def test_incoming_convention_fails_hankel_pin():
    # Planted mistake: flipping the sign of the stretching makes waves grow in
    # the layer; the field no longer matches the outgoing Hankel function.
    n, omega = 127, 2 * np.pi * 4
    h = 1.0 / (n + 1)
    npml = int(round(0.2 / h))
    st = _stencil(n, omega, npml)
    # rebuild with sigma -> -sigma, i.e. s -> conj(s)
    st_bad = assemble.stencil(W.constant_medium(n), omega, npml, C=-pml.DEFAULT_C)
    f = W.gaussian_source(n, (0.5, 0.5)).ravel()
    ur, r = hankel.gaussian_field(n, omega, (0.5, 0.5))
    mask = (r >= 0.1) & (r <= 0.3)
    good = direct.solve_sparse(st, f).reshape(n, n)
    bad = direct.solve_sparse(st_bad, f).reshape(n, n)
    e_good = np.linalg.norm(good[mask] - ur[mask]) / np.linalg.norm(ur[mask])
    e_bad = np.linalg.norm(bad[mask] - ur[mask]) / np.linalg.norm(ur[mask])
    assert e_good < 1e-2 and e_bad > 0.2


def test_dropped_edge_term_fails_fast_diagonalization_pin():
    # Planted mistake: a centre coefficient that forgets the north edge.
    n, npml, omega = 31, 6, 2 * np.pi * 4
    st = _stencil(n, omega, npml)
    D_bad = st.D + st.N
    st_bad = assemble.Stencil(n=st.n, omega=st.omega, h=st.h, W=st.W, E=st.E, S=st.S, N=st.N,
                              D=D_bad, s1s2=st.s1s2, c=st.c)
    f = W.gaussian_source(n, (0.5, 0.5)).ravel()
    u_fd = fastdiag.solve_constant(n, omega, npml, 1.0, f)
    ok = direct.solve_sparse(st, f)
    bad = direct.solve_sparse(st_bad, f)
    assert np.linalg.norm(ok - u_fd) / np.linalg.norm(u_fd) < 1e-10
    assert np.linalg.norm(bad - u_fd) / np.linalg.norm(u_fd) > 1e-3


# ---------------------------------------------------------------- other boundaries and directions

def test_per_side_layers_reduce_to_the_symmetric_layer_and_mirror():
    n = 31
    c = W.random_field_medium(n, 17)
    om = 2 * np.pi * 3
    a = assemble.stencil(c, om, 5)
    b = assemble.stencil(c, om, (5, 5, 5, 5))
    for f in ("W", "E", "S", "N", "D", "s1s2"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    # reflecting the grid in x2 swaps the two x2 widths (to rounding of the node positions)
    st = assemble.stencil(c, om, (3, 7, 2, 6))
    sr = assemble.stencil(c[::-1].copy(), om, (3, 7, 6, 2))
    np.testing.assert_allclose(sr.D, st.D[::-1], rtol=1e-12)
    np.testing.assert_allclose(sr.N, st.S[::-1], rtol=1e-12)
    np.testing.assert_allclose(sr.W, st.W[::-1], rtol=1e-12)
    # a side of width 0 has no layer: the stretching is 1 there
    sig = pml.sigma_sides(np.linspace(0, 1, 41), 0.0, 0.25, 9.0)
    assert np.all(sig[:30] == 0) and sig[-1] == pytest.approx(9.0 / 0.25)


def _mode(n, p, omega):
    # u = sin(p pi x1) exp(i kappa x2) solves the 5-point equation with c = 1 and
    # no absorbing layer exactly when (2 - 2cos(p pi h) + 2 - 2cos(kappa h)) / h^2 = omega^2
    h = 1.0 / (n + 1)
    ck = 1.0 - 0.5 * h * h * (omega ** 2 - (2 - 2 * np.cos(p * np.pi * h)) / h ** 2)
    kappa = np.arccos(ck) / h
    x = h * np.arange(0, n + 2)
    U = np.sin(p * np.pi * x)[None, :] * np.exp(1j * kappa * x)[:, None]   # [j, i] incl. boundary
    return U, kappa


def test_dirichlet_data_reproduce_an_exact_discrete_mode():
    n, p, om = 31, 2, 2 * np.pi * 2
    U, kappa = _mode(n, p, om)
    st = assemble.stencil(W.constant_medium(n), om, 0)
    g = assemble.dirichlet_forcing(st, "x2=0", U[0, 1:-1]) + assemble.dirichlet_forcing(st, "x2=1", U[-1, 1:-1])
    u = direct.solve_sparse(st, g)
    np.testing.assert_allclose(u, U[1:-1, 1:-1].ravel(), rtol=0, atol=1e-10)
    # the same mode turned by 90 degrees, data on the x1 edges
    Ut = U.T
    g = assemble.dirichlet_forcing(st, "x1=0", Ut[1:-1, 0]) + assemble.dirichlet_forcing(st, "x1=1", Ut[1:-1, -1])
    np.testing.assert_allclose(direct.solve_sparse(st, g), Ut[1:-1, 1:-1].ravel(), rtol=0, atol=1e-10)
    # planted mistake: dropping the top edge's data is caught
    g_bad = assemble.dirichlet_forcing(st, "x2=0", U[0, 1:-1])
    assert np.max(np.abs(direct.solve_sparse(st, g_bad) - U[1:-1, 1:-1].ravel())) > 1e-2


@pytest.mark.parametrize("direction", assemble.DIRECTIONS)
def test_frame_stencil_is_the_relabelled_operator(direction):
    n = 11
    st = assemble.stencil(W.random_field_medium(n, 23), 2 * np.pi * 1.5, (1, 2, 3, 2))
    A = assemble.matrix(st).toarray()
    idx = np.arange(n * n).reshape(n, n)                    # natural flat index at [j, i]
    perm = np.ascontiguousarray(assemble.to_frame(idx, direction)).ravel()   # frame position -> natural index
    Af = assemble.matrix(assemble.permuted(st, direction)).toarray()
    np.testing.assert_array_equal(Af, A[np.ix_(perm, perm)])
    back = assemble.from_frame(assemble.to_frame(idx, direction), direction)
    np.testing.assert_array_equal(back, idx)


@pytest.mark.parametrize("direction", assemble.DIRECTIONS)
def test_exact_sweep_in_every_direction_is_the_inverse(direction):
    n = 15
    st = assemble.stencil(W.random_field_medium(n, 29), 2 * np.pi * 2, (2, 3, 1, 4))
    rng = np.random.default_rng(4)
    f = rng.standard_normal((2, n * n)) + 1j * rng.standard_normal((2, n * n))
    u, _ = sweep.solve_direction(st, f, direction)
    np.testing.assert_allclose(u, direct.solve_dense(st, f), rtol=0, atol=1e-10 * np.abs(u).max())


# ---------------------------------------------------------------- absorbing boundary condition

def _reflection(n, p, om, monkey=None):
    """Solve with u = sin(p pi x1) on x2 = 0, zero on the x1 sides and the
    absorbing condition on x2 = 1 (c = 1, no layers).  The solution is a
    combination of the two exact discrete modes sin(p pi x1) e^{+-i kappa x2};
    returns their ratio at x2 = 1 (the reflection coefficient) and the misfit
    of that two-mode form."""
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    st = assemble.stencil(W.constant_medium(n), om, 0, abc=("x2=1",))
    b = np.sin(p * np.pi * x)
    u = direct.solve_sparse(st, assemble.dirichlet_forcing(st, "x2=0", b)).reshape(n, n)
    U = u @ b / (b @ b)
    lam = (2 - 2 * np.cos(p * np.pi * h)) / h ** 2
    kap = np.arccos(1 - 0.5 * h * h * (om ** 2 - lam)) / h
    M = np.stack([np.exp(1j * kap * x), np.exp(-1j * kap * x)], 1)
    (A, B), *_ = np.linalg.lstsq(M, U, rcond=None)
    fit = np.abs(M @ np.array([A, B]) - U).max() / np.abs(U).max()
    return B * np.exp(-1j * kap) / (A * np.exp(1j * kap)), fit


def _engquist_majda(p, om, first_order=False):
    # plane wave e^{i(kx x1 + ky x2)} against du/dn = i k u + (i/(2k)) u_tt:
    # r = (cos t - 1 + sin^2 t / 2) / (cos t + 1 - sin^2 t / 2)
    s2 = (p * np.pi / om) ** 2
    ct = np.sqrt(1 - s2)
    q = 1.0 if first_order else 1 - s2 / 2
    return (ct - q) / (ct + q)


@pytest.mark.parametrize("p", [3, 6])
def test_absorbing_condition_reflection_converges_to_the_continuous_one(p):
    om = 2 * np.pi * 4
    R2 = _engquist_majda(p, om)
    errs = []
    for n in (63, 127, 255):
        r, fit = _reflection(n, p, om)
        assert fit <= 1e-10                       # exact separable solution: corners close on zero values
        errs.append(abs(r - R2))
    assert errs[0] / errs[1] >= 1.8 and errs[1] / errs[2] >= 1.8
    assert errs[-1] <= 5e-3
    if p == 6:                                    # 49 degrees: far from the first-order condition
        assert abs(r - _engquist_majda(p, om, first_order=True)) > 0.1


def test_absorbing_condition_near_normal_incidence_converges_at_second_order():
    om = 2 * np.pi * 4                       # p = 1: 7 degrees, where the tangential term is negligible
    e = [abs(_reflection(n, 1, om)[0] - _engquist_majda(1, om)) for n in (63, 127, 255)]
    assert e[0] / e[1] >= 3.5 and e[1] / e[2] >= 3.5


def test_flipped_tangential_term_is_caught(monkeypatch):
    # Planted mistake: the tangential term with the wrong sign.
    good = assemble.abc_g
    monkeypatch.setattr(assemble, "abc_g", lambda k, h: -good(k, h))
    om = 2 * np.pi * 4
    r, _ = _reflection(255, 6, om)
    assert abs(r - _engquist_majda(6, om)) > 0.1


def test_absorbing_condition_keeps_symmetry_and_absorbs_a_point_source():
    import scipy.special as sps
    n = 255
    om = 2 * np.pi * 8
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    X, Y = np.meshgrid(x, x)
    f = W.gaussian_source(n, (0.5, 0.5)).ravel()
    r = np.hypot(X - 0.5, Y - 0.5)
    ref = -(1j / 4) * np.exp(-(om * 1.5 * h) ** 2 / 2) * sps.hankel1(0, om * np.maximum(r, 1e-9))
    ann = (r >= 0.1) & (r <= 0.3)
    err = {}
    for abc in (assemble.EDGES, ()):
        st = assemble.stencil(W.constant_medium(n), om, 0, abc=abc)
        A = assemble.matrix(st)
        assert abs(A - A.T).max() == 0
        u = direct.solve_sparse(st, f).reshape(n, n)
        err[abc] = np.linalg.norm(u[ann] - ref[ann]) / np.linalg.norm(ref[ann])
    assert err[assemble.EDGES] <= 0.06 and err[()] >= 0.5
    # mixed sides: absorbing condition beside layers and zero Dirichlet sides
    st = assemble.stencil(W.random_field_medium(31, 3), 2 * np.pi * 3, (0, 4, 0, 0), abc=("x1=0", "x2=1"))
    A = assemble.matrix(st)
    assert abs(A - A.T).max() == 0
    U = np.random.default_rng(2).standard_normal((3, 31 * 31)) + 0j
    np.testing.assert_allclose(assemble.apply(st, U), (A @ U.T).T, rtol=0, atol=1e-10 * np.abs(A).max())
