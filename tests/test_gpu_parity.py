"""GPU parity of the HIP sweeping solver against the FP64 CPU oracle.

Every test calls the C-ABI library through the Python binding; the oracle
side is computed on the CPU from the same seeded inputs.  Tolerances:
* stencil (FP64 on both sides, different rounding order): 1e-13 relative;
* uncompressed factors (dense Schur, or H-blocks with rank >= block size and
  no truncation), complex128: the sweep is the exact inverse, 1e-10;
* compressed factors: the GMRES solution is compared with u = A^{-1} f;
  complex128 sweep with GMRES tol 1e-12 -> 1e-8, complex64 sweep with FP64
  GMRES tol 1e-10 -> 1e-5 (the metric's stated bounds are 1e-6 / 1e-5).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import assemble, direct, gradient, sweep  # noqa: E402
import workloads as W  # noqa: E402
from parity import assert_close  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _Solver():
    from paper_1007_4290_amd.solver import Solver
    return Solver


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), device=DEV)


def _problem(n, freq, npml, medium="grf", seed=1):
    c = W.random_field_medium(n, seed) if medium == "grf" else (
        W.lens_medium(n) if medium == "lens" else W.constant_medium(n))
    return c, 2 * np.pi * freq, npml


# ----------------------------------------------------------------- stencil

@pytest.mark.parametrize("n", [31, 63, 255])
def test_stencil_matches_oracle(n):
    _need_gpu()
    c, omega, npml = _problem(n, n / 8, max(2, n // 16))
    s = _Solver()(c, omega, npml)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((2, n * n)) + 1j * rng.standard_normal((2, n * n))
    y = s.stencil(_t(x)).cpu().numpy()
    st = assemble.stencil(c, omega, npml)
    assert_close(y, assemble.apply(st, x), 1e-13, "stencil")


# ----------------------------------------------------------------- exact factors

@pytest.mark.parametrize("n,dense,leaf,rank", [
    (7, True, 0, 2),      # dense Schur, tiny (padded 7 -> 8)
    (15, False, 4, 8),    # H-blocks, 2 levels, rank 8 = largest block -> exact
    (23, False, 4, 16),   # ragged: 23 -> 32 with 9 padding unknowns, 3 levels
    (31, False, 4, 16),   # 3 levels, rank 16 = largest block -> exact
])
def test_uncompressed_sweep_is_exact_inverse(n, dense, leaf, rank):
    _need_gpu()
    c, omega, npml = _problem(n, max(1.0, n / 8), max(1, n // 8))
    s = _Solver()(c, omega, npml, dense=dense, leaf=leaf or 16, rank=rank, rank_tol=0.0).factor()
    st = assemble.stencil(c, omega, npml)
    f = W.gaussian_source(n, (0.5, 0.5)).reshape(1, -1)
    rng = np.random.default_rng(3)
    f = np.vstack([f, rng.standard_normal((1, n * n)) + 1j * rng.standard_normal((1, n * n))])
    u = s.apply(_t(f)).cpu().numpy()
    ue = direct.solve_sparse(st, f)
    for k in range(2):
        assert_close(u[k], ue[k], 1e-10, f"rhs {k}")


def test_dense_schur_helm63_one_gmres_iteration():
    _need_gpu()
    wl = W.get("helm63_dense_c1")
    c = wl.velocity()
    s = _Solver()(c, wl.omega, wl.pml, dense=True).factor()
    f = wl.sources()
    u, its, res = s.solve(_t(f), tol=1e-12)
    st = assemble.stencil(c, wl.omega, wl.pml)
    ue = direct.solve_sparse(st, f)
    assert its == [1]
    assert res[0] <= 1e-12
    assert_close(u.cpu().numpy()[0], ue[0], 1e-10, "solution")
    # the factors equal the oracle's exact sweep: compare M f
    T = sweep.factor(st)
    mf = s.apply(_t(f)).cpu().numpy()
    assert_close(mf[0], sweep.solve(st, T, f[0]), 1e-10, "M f")


# ----------------------------------------------------------------- compressed factors

@pytest.fixture(scope="module")
def helm255():
    wl = W.get("helm255_grf")
    c = wl.velocity()
    st = assemble.stencil(c, wl.omega, wl.pml)
    f = wl.sources()
    ue = direct.solve_sparse(st, f)
    return wl, c, st, f, ue


def test_helm255_c128_solution(helm255):
    _need_gpu()
    wl, c, st, f, ue = helm255
    s = _Solver()(c, wl.omega, wl.pml, leaf=16, rank=8, rank_tol=1e-6, precision="c128").factor()
    u, its, res = s.solve(_t(f), tol=1e-12)
    assert res[0] <= 1e-12
    assert its[0] <= 10
    assert_close(u.cpu().numpy()[0], ue[0], 1e-8, "c128")
    assert direct.relative_residual(st, u.cpu().numpy()[0], f[0]) < 1e-11
    info = s.plan_info()
    assert info["n_p"] == 256 and info["levels"] == 4


def test_helm255_c64_solution(helm255):
    _need_gpu()
    wl, c, st, f, ue = helm255
    s = _Solver()(c, wl.omega, wl.pml, leaf=16, rank=8, rank_tol=1e-6, precision="c64").factor()
    u, its, res = s.solve(_t(f), tol=1e-10)
    assert res[0] <= 1e-10
    assert its[0] <= 15
    assert_close(u.cpu().numpy()[0], ue[0], 1e-5, "c64")
    # metric setting: residual 1e-6
    u6, its6, res6 = s.solve(_t(f), tol=1e-6)
    assert res6[0] <= 1e-6
    assert direct.relative_residual(st, u6.cpu().numpy()[0], f[0]) <= 1.0001e-6


def test_multiple_right_hand_sides_match_single_solves():
    _need_gpu()
    c, omega, npml = _problem(127, 16, 12)
    s = _Solver()(c, omega, npml, leaf=16, rank=8, rank_tol=1e-6).factor()
    pos = W.uniform_source_positions(127, 12, 3, seed=9)
    F = np.stack([W.gaussian_source(127, p).ravel() for p in pos])
    U, its, res = s.solve(_t(F), tol=1e-11)
    st = assemble.stencil(c, omega, npml)
    ue = direct.solve_sparse(st, F)
    for k in range(3):
        assert res[k] <= 1e-11
        assert_close(U[k].cpu().numpy(), ue[k], 1e-8, f"rhs {k}")
        u1, _, _ = s.solve(_t(F[k]), tol=1e-11)
        assert_close(u1.cpu().numpy(), ue[k], 1e-8, f"single {k}")


def test_apply_batch_rows_are_independent():
    _need_gpu()
    c, omega, npml = _problem(63, 8, 8)
    s = _Solver()(c, omega, npml, leaf=8, rank=8).factor()
    rng = np.random.default_rng(5)
    F = rng.standard_normal((4, 63 * 63)) + 1j * rng.standard_normal((4, 63 * 63))
    U = s.apply(_t(F)).cpu().numpy()
    for k in range(4):
        assert_close(s.apply(_t(F[k])).cpu().numpy(), U[k], 1e-14, f"rhs {k}")


@pytest.mark.parametrize("precision,n,leaf,tol", [
    ("c64", 127, 16, 2e-5),     # matrix-core products (complex64, 4 right-hand sides per workgroup)
    ("c128", 127, 16, 1e-14),   # vector products, same summation order as one per workgroup
    ("c64", 255, 32, 2e-5),
])
def test_grouped_sweep_matches_single_rhs_sweep(precision, n, leaf, tol):
    # rhs_group = 4 loads each layer once for 4 right-hand sides; 6 fields
    # make one full and one partial group (the last two slots idle)
    _need_gpu()
    c, omega, npml = _problem(n, (n + 1) / 8, 12)
    one = _Solver()(c, omega, npml, leaf=leaf, rank=8, rank_tol=1e-6, precision=precision, rhs_group=1).factor()
    grp = _Solver()(c, omega, npml, leaf=leaf, rank=8, rank_tol=1e-6, precision=precision, rhs_group=4).factor()
    rng = np.random.default_rng(n)
    F = rng.standard_normal((6, n * n)) + 1j * rng.standard_normal((6, n * n))
    a = one.apply(_t(F)).cpu().numpy()
    b = grp.apply(_t(F)).cpu().numpy()
    for k in range(6):
        assert_close(b[k], a[k], tol, f"rhs {k}")


def test_grouped_sweep_solution_matches_oracle():
    _need_gpu()
    c, omega, npml = _problem(255, 32, 16)
    s = _Solver()(c, omega, npml, leaf=16, rank=8, rank_tol=1e-6, precision="c64", rhs_group=4).factor()
    pos = W.uniform_source_positions(255, 16, 5, seed=12)
    F = np.stack([W.gaussian_source(255, p).ravel() for p in pos])
    U, its, res = s.solve(_t(F), tol=1e-10)
    assert max(res) <= 1e-10
    Ue = direct.SparseLU(assemble.stencil(c, omega, npml)).solve(F)
    for k in range(5):
        assert_close(U[k].cpu().numpy(), Ue[k], 1e-5, f"source {k}")


# ----------------------------------------------------------------- gradient

def test_gradient_matches_oracle_adjoint():
    _need_gpu()
    n, npml = 63, 6
    omega = 2 * np.pi * 6
    c0 = W.constant_medium(n)
    c_true = W.random_field_medium(n, 5)
    F = np.stack([W.gaussian_source(n, p).ravel() for p in W.bottom_row_sources(n, npml, 4, margin=4)])
    rec = W.top_row_receivers(n, npml, 24, margin=4)
    _, _, U_true = gradient.forward(c_true, omega, npml, F)
    data = U_true[:, rec]
    J_ref, g_ref = gradient.adjoint_gradient(c0, omega, npml, F, rec, data)
    from paper_1007_4290_amd.solver import helmholtz_solve
    c_t = _t(c0).requires_grad_(True)
    u = helmholtz_solve(c_t, _t(F), omega, npml, tol=1e-12, leaf=8, rank=8, rank_tol=1e-8)
    r = u[:, torch.as_tensor(rec, device=DEV)] - _t(data)
    J = 0.5 * (r.abs() ** 2).sum()
    J.backward()
    assert float(J.detach()) == pytest.approx(J_ref, rel=1e-8)
    assert_close(c_t.grad.cpu().numpy(), g_ref, 1e-7, "dJ/dc")


def test_adjoint_entry_point_matches_oracle():
    # hsweep_solve_adjoint: mu = A^{-1} conj(g) and grad_f = conj(mu), both
    # computed in the library, against the oracle's adjoint fields
    _need_gpu()
    n, npml = 63, 6
    omega = 2 * np.pi * 6
    c0 = W.random_field_medium(n, 31)
    F = np.stack([W.gaussian_source(n, p).ravel() for p in W.bottom_row_sources(n, npml, 3, margin=4)])
    rec = W.top_row_receivers(n, npml, 20, margin=4)
    data = np.full((3, rec.size), 0.01 - 0.02j)
    J_ref, _, U_ref, Mu_ref = gradient.adjoint_state(c0, omega, npml, F, rec, data)
    G = np.zeros_like(U_ref)
    G[:, rec] = U_ref[:, rec] - data
    s = _Solver()(c0, omega, npml, leaf=8, rank=8, rank_tol=1e-8, precision="c64").factor()
    mu, gf, its, res = s.solve_adjoint(_t(G), tol=1e-12, want_grad_f=True)
    assert max(res) <= 1e-12
    for k in range(3):
        assert_close(mu[k].cpu().numpy(), Mu_ref[k], 1e-8, f"mu {k}")
        assert_close(gf[k].cpu().numpy(), np.conj(Mu_ref[k]), 1e-8, f"grad_f {k}")
    mu2, gf2, _, _ = s.solve_adjoint(_t(G[0]), tol=1e-12)
    assert gf2 is None
    assert_close(mu2.cpu().numpy(), Mu_ref[0], 1e-8, "single")


def test_workspace_bytes_cover_the_factor_store():
    _need_gpu()
    c, omega, npml = _problem(127, 16, 8)
    s = _Solver()(c, omega, npml, leaf=16, rank=8, rank_tol=1e-6, precision="c64")
    fb1, sb1 = s.workspace_bytes(1)
    fb4, sb4 = s.workspace_bytes(4)
    s.factor()
    store = s.plan_info()["factor_bytes"]
    assert store > 0 and fb1 >= store and fb1 == fb4
    assert sb4 > sb1 > 0
    # the 41 + 40 Krylov fields of one right-hand side at restart 40
    assert sb1 >= 81 * 127 * 127 * 16


# ----------------------------------------------------------------- batch API and errors

def test_batch_entry_points_mixed_sizes():
    _need_gpu()
    from paper_1007_4290_amd.solver import factor_batch, solve_batch
    Solver = _Solver()
    sizes = [31, 63, 31]
    solvers, fs, refs = [], [], []
    for k, n in enumerate(sizes):
        c, omega, npml = _problem(n, n / 8 + 0.5, 4, seed=100 + k)
        solvers.append(Solver(c, omega, npml, leaf=8, rank=8))
        f = W.gaussian_source(n, (0.5, 0.5)).ravel()
        fs.append(_t(f))
        refs.append(direct.solve_sparse(assemble.stencil(c, omega, npml), f))
    factor_batch(solvers)
    us, its, res = solve_batch(solvers, fs, tol=1e-11)
    for u, ref, rr in zip(us, refs, res):
        assert rr <= 1e-11
        assert_close(u.cpu().numpy(), ref, 1e-8, "batch")


def test_error_codes_on_device():
    _need_gpu()
    from paper_1007_4290_amd import _lib
    Solver = _Solver()
    c, omega, npml = _problem(31, 4, 4)
    s = Solver(c, omega, npml, leaf=8, rank=8)
    f = _t(W.gaussian_source(31, (0.5, 0.5)).ravel())
    with pytest.raises(_lib.HsweepError) as e:
        s.apply(f)
    assert e.value.code == _lib.ESTATE
    s.factor()
    u, its, res = s.solve(f, tol=1e-14, maxit=1, allow_noconv=True)
    assert its == 1 and res > 1e-14
    with pytest.raises(_lib.HsweepError) as e:
        s.solve(f, tol=1e-14, maxit=1)
    assert e.value.code == _lib.ENOCONV


def test_factor_profile_gives_the_same_factor():
    # the per-kernel timed factorization (plain launches) and the graph replay
    # must produce identical factors
    _need_gpu()
    c, omega, npml = _problem(127, 16, 8)
    s = _Solver()(c, omega, npml, leaf=16, rank=8, rank_tol=1e-6, precision="c64")
    f = _t(W.gaussian_source(127, (0.5, 0.5)).reshape(1, -1))
    s.factor()
    a = s.apply(f).cpu().numpy()
    s.factor()                              # graph replay
    b = s.apply(f).cpu().numpy()
    prof = s.profile_factor()
    c2 = s.apply(f).cpu().numpy()
    assert np.array_equal(a, b) and np.array_equal(a, c2)
    assert prof["layers"] == 127 and prof["layer_ms"] > 0 and prof["wood_ms"] > 0
