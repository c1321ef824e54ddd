"""The 3D face-by-face sweep on the GPU (Sec. 4) against the FP64 oracle:
the 7-point operator, untruncated strongly admissible face factors (the
exact inverse), and rank-2 face factors inside FP64 GMRES (the paper's 3D
setting).  The same cases run on the CPU through the kernel emulation of
tests/test_strong3d_emulated.py."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

from oracle import threed as T3  # noqa: E402
from parity import assert_close  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), device=DEV)


def _medium(n, seed):
    return 1 + 0.3 * np.random.default_rng(seed).random((n, n, n))


def _centre_source(n):
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    s = 1.5 * h
    g = np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5
    return g.ravel().astype(complex)


def _Solver3():
    from paper_1007_4290_amd.solver import Solver3
    return Solver3


def test_operator_equals_the_oracle():
    _need_gpu()
    n, om, pml = 7, 2 * np.pi * 1.5, 2
    c = _medium(n, 1)
    F = np.random.default_rng(2).standard_normal((2, n ** 3)) + 1j * np.random.default_rng(3).standard_normal((2, n ** 3))
    s = _Solver3()(c, om, pml, leaf=4, rank=16, rank_tol=0.0)
    assert_close(s.stencil(_t(F)).cpu().numpy(), T3.apply(T3.stencil(c, om, pml), F), 1e-13, "operator")


@pytest.mark.parametrize("n", [7, 8])
def test_untruncated_face_factors_are_the_exact_inverse(n):
    _need_gpu()
    om, pml = 2 * np.pi * 1.5, 2
    c = _medium(n, n)
    rng = np.random.default_rng(5)
    F = rng.standard_normal((2, n ** 3)) + 1j * rng.standard_normal((2, n ** 3))
    s = _Solver3()(c, om, pml, leaf=4, rank=64, rank_tol=0.0).factor()
    info = s.plan_info()
    assert info["levels"] == 4 and info["factor_bytes"] > 0
    U = s.apply(_t(F)).cpu().numpy()
    Ue = spla.spsolve(T3.matrix(T3.stencil(c, om, pml)).tocsc(), F.T).T
    for k in range(2):
        assert_close(U[k], Ue[k], 1e-10, f"n = {n} rhs {k}")


def test_rank_two_face_factors_precondition_gmres_to_the_solution():
    _need_gpu()
    n, om, pml = 15, 2 * np.pi * 2, 3
    c = _medium(n, 13)
    f = _centre_source(n)
    s = _Solver3()(c, om, pml, leaf=16, rank=2, rank_tol=1e-6).factor()
    u, its, res = s.solve(_t(f), tol=1e-10, maxit=50)
    assert res <= 1e-10 and its <= 10
    ue = spla.spsolve(T3.matrix(T3.stencil(c, om, pml)).tocsc(), f)
    assert_close(u.cpu().numpy(), ue, 1e-8, "3D rank 2")
    print(f"3D rank-2 face factors, n = 15: {its} GMRES iterations")


def test_3d_context_rejects_weak_or_complex64_faces():
    _need_gpu()
    from paper_1007_4290_amd import _lib
    import ctypes
    n = 7
    s = _Solver3()(_medium(n, 1), 2 * np.pi, 2)
    o = _lib.default_opts()
    o.admissibility = _lib.ADMISSIBILITY["weak"]
    assert _lib.load().hsweep3_set_opts(s._ctx, ctypes.byref(o)) == _lib.EINVAL
    o.admissibility = _lib.ADMISSIBILITY["strong"]
    o.precision = _lib.C64
    assert _lib.load().hsweep3_set_opts(s._ctx, ctypes.byref(o)) == _lib.EINVAL
    z = _t(np.zeros(n ** 3, complex))
    with pytest.raises(_lib.HsweepError) as e:
        s.apply(z)                                   # before factor
    assert e.value.code == _lib.ESTATE
