"""Python front end of the HIP sweeping solver.

PyTorch is used for device memory and streams only: fields are complex128
CUDA tensors of shape (nrhs, n*n) (or (n*n,)), in the grid ordering of
include/hsweep.h, and every computation is a call into libhsweep.so.
"""
import ctypes

import numpy as np
import torch

from . import _lib

_PREC = {"c128": _lib.C128, "c64": _lib.C64}


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _as_fields(x, n):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("fields must be CUDA tensors")
    if x.dtype != torch.complex128:
        raise TypeError("fields must be complex128")
    single = x.dim() == 1
    x2 = x.reshape(1, -1) if single else x.reshape(x.shape[0], -1)
    if x2.shape[1] != n * n:
        raise ValueError(f"each field must have n*n = {n * n} entries")
    return x2.contiguous(), single


class Solver:
    """Sweeping-preconditioned GMRES solver for one medium and frequency.

    c: velocity (n x n, indexed [j-1, i-1]) as numpy array or tensor;
    omega: angular frequency; pml: absorbing-layer width in grid points.
    Options: leaf, rank, rank_tol, precision ("c128" | "c64"), dense,
    restart, pml_C, rhs_group (right-hand sides per sweep workgroup:
    0 automatic, 1 or 4), direction ("+x2", "-x2", "+x1", "-x1"),
    pml_sides (layer widths on the sides x1=0, x1=1, x2=0, x2=1; 0 for a
    zero Dirichlet side, "abc" for the second-order absorbing boundary
    condition; default: `pml` on every side), admissibility ("weak" or
    "strong"; strong runs in complex128, one context at a time).
    """

    def __init__(self, c, omega, pml, leaf=16, rank=8, rank_tol=1e-6, precision="c128", dense=False,
                 restart=40, pml_C=20.0, rhs_group=0, direction="+x2", pml_sides=None, admissibility="weak"):
        lib = _lib.load()
        if isinstance(c, torch.Tensor):
            c_t = c.detach().to(torch.float64).contiguous()
        else:
            c_t = torch.as_tensor(np.ascontiguousarray(c, dtype=np.float64))
        n = int(c_t.shape[0])
        if c_t.dim() != 2 or c_t.shape[1] != n:
            raise ValueError("c must be a square (n, n) array")
        self.n = n
        self.omega = float(omega)
        self.pml = int(pml)
        self._c = c_t
        self._ctx = ctypes.c_void_p()
        _lib.check(lib.hsweep_setup(ctypes.c_void_p(c_t.data_ptr()), self.omega, self.pml, n,
                                    ctypes.byref(self._ctx)))
        o = _lib.default_opts()
        o.leaf, o.rank, o.rank_tol = int(leaf), int(rank), float(rank_tol)
        o.pml_C, o.precision, o.dense, o.restart = float(pml_C), _PREC[precision], int(bool(dense)), int(restart)
        o.rhs_group = int(rhs_group)
        o.direction = _lib.DIRECTIONS[direction]
        sides = (-1, -1, -1, -1) if pml_sides is None else \
            tuple(_lib.SIDE_ABC if (isinstance(v, str) and v == "abc") else int(v) for v in pml_sides)
        if len(sides) != 4:
            raise ValueError("pml_sides holds the widths of the sides x1=0, x1=1, x2=0, x2=1")
        for k in range(4):
            o.pml_sides[k] = sides[k]
        o.admissibility = _lib.ADMISSIBILITY[admissibility]
        _lib.check(lib.hsweep_set_opts(self._ctx, ctypes.byref(o)))
        self.precision = precision
        self.factored = False

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            _lib.load().hsweep_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- plan --------------------------------------------------------------
    def plan_info(self):
        npad, lev, fb = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _lib.check(_lib.load().hsweep_plan_info(self._ctx, ctypes.byref(npad), ctypes.byref(lev), ctypes.byref(fb)))
        return {"n_p": npad.value, "levels": lev.value, "factor_bytes": fb.value}

    def timings(self):
        out = (ctypes.c_double * 5)()
        _lib.check(_lib.load().hsweep_timings(self._ctx, out, 5))
        return {"factor_ms": out[0], "sweep_ms": out[1], "stencil_ms": out[2], "krylov_ms": out[3],
                "applies": int(out[4])}

    def profile_factor(self, stream=None):
        """Factor with HIP events around each kernel class; returns the total
        milliseconds of the layer kernels and of the Woodbury kernels and the
        number of layers (one layer kernel launch each)."""
        out = (ctypes.c_double * 3)()
        _lib.check(_lib.load().hsweep_factor_profile(self._ctx, _stream_ptr(stream), out, 3))
        self.factored = True
        return {"layer_ms": out[0], "wood_ms": out[1], "layers": int(out[2])}

    # -- operations --------------------------------------------------------
    def factor(self, stream=None):
        _lib.check(_lib.load().hsweep_factor(self._ctx, _stream_ptr(stream)))
        self.factored = True
        return self

    def apply(self, f, stream=None):
        """u = M f (one sweep of the preconditioner)."""
        f2, single = _as_fields(f, self.n)
        u = torch.empty_like(f2)
        _lib.check(_lib.load().hsweep_apply(self._ctx, ctypes.c_void_p(f2.data_ptr()),
                                            ctypes.c_void_p(u.data_ptr()), f2.shape[0], _stream_ptr(stream)))
        return u[0] if single else u

    def stencil(self, x, stream=None):
        """y = A x with the FP64 5-point operator."""
        x2, single = _as_fields(x, self.n)
        y = torch.empty_like(x2)
        _lib.check(_lib.load().hsweep_stencil(self._ctx, ctypes.c_void_p(x2.data_ptr()),
                                              ctypes.c_void_p(y.data_ptr()), x2.shape[0], _stream_ptr(stream)))
        return y[0] if single else y

    def solve(self, f, tol=1e-6, maxit=200, stream=None, allow_noconv=False):
        """Flexible GMRES; returns (u, iterations, relative residuals)."""
        f2, single = _as_fields(f, self.n)
        k = f2.shape[0]
        u = torch.empty_like(f2)
        its = (ctypes.c_int * k)()
        res = (ctypes.c_double * k)()
        rc = _lib.load().hsweep_solve(self._ctx, ctypes.c_void_p(f2.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                      k, float(tol), int(maxit), its, res, _stream_ptr(stream))
        if not (allow_noconv and rc == _lib.ENOCONV):
            _lib.check(rc)
        its_l, res_l = list(its), list(res)
        if single:
            return u[0], its_l[0], res_l[0]
        return u, its_l, res_l

    def solve_adjoint(self, g, tol=1e-6, maxit=200, want_grad_f=False, stream=None, allow_noconv=False):
        """mu = A^{-1} conj(g) (and grad_f = conj(mu) if asked), computed in the
        library; returns (mu, grad_f or None, iterations, relative residuals)."""
        g2, single = _as_fields(g, self.n)
        k = g2.shape[0]
        mu = torch.empty_like(g2)
        gf = torch.empty_like(g2) if want_grad_f else None
        its = (ctypes.c_int * k)()
        res = (ctypes.c_double * k)()
        rc = _lib.load().hsweep_solve_adjoint(self._ctx, ctypes.c_void_p(g2.data_ptr()), ctypes.c_void_p(mu.data_ptr()),
                                              ctypes.c_void_p(gf.data_ptr() if gf is not None else None), k,
                                              float(tol), int(maxit), its, res, _stream_ptr(stream))
        if not (allow_noconv and rc == _lib.ENOCONV):
            _lib.check(rc)
        if single:
            return mu[0], (gf[0] if gf is not None else None), its[0], res[0]
        return mu, gf, list(its), list(res)

    def workspace_bytes(self, nrhs=1):
        """Device bytes the library allocates: (factorization, solve of nrhs right-hand sides)."""
        fb, sb = ctypes.c_size_t(), ctypes.c_size_t()
        _lib.check(_lib.load().hsweep_workspace_bytes(self._ctx, int(nrhs), ctypes.byref(fb), ctypes.byref(sb)))
        return fb.value, sb.value

    def dirichlet_forcing(self, edge, b, f, stream=None):
        """f - (coupling to the boundary) * b on the row next to `edge`
        ("x1=0", "x1=1", "x2=0", "x2=1"): Dirichlet data b moved to the
        right-hand side.  b: complex128 CUDA tensor (nrhs, n) or (n,); f is
        not modified, the result is returned."""
        f2, single = _as_fields(f, self.n)
        out = f2.clone()
        if not isinstance(b, torch.Tensor) or not b.is_cuda or b.dtype != torch.complex128:
            raise TypeError("b must be a complex128 CUDA tensor")
        b2 = b.reshape(out.shape[0], self.n).contiguous()
        _lib.check(_lib.load().hsweep_dirichlet_forcing(self._ctx, _lib.EDGES[edge], ctypes.c_void_p(b2.data_ptr()),
                                                        ctypes.c_void_p(out.data_ptr()), out.shape[0],
                                                        _stream_ptr(stream)))
        return out[0] if single else out

    def grad_c(self, u, mu, stream=None):
        """sum_k Re(mu_k u_k 2 omega^2 / ((s1 s2) c^3)) as an (n, n) float64 tensor."""
        u2, _ = _as_fields(u, self.n)
        m2, _ = _as_fields(mu, self.n)
        if u2.shape != m2.shape:
            raise ValueError("u and mu must have the same shape")
        g = torch.empty((self.n, self.n), dtype=torch.float64, device=u2.device)
        _lib.check(_lib.load().hsweep_grad_c(self._ctx, ctypes.c_void_p(u2.data_ptr()),
                                             ctypes.c_void_p(m2.data_ptr()), u2.shape[0],
                                             ctypes.c_void_p(g.data_ptr()), _stream_ptr(stream)))
        return g


class Solver3:
    """Face-by-face sweeping-preconditioned GMRES for the 3D problem (Sec. 4).

    c: velocity of shape (n, n, n), indexed [k-1, j-1, i-1] (x3, x2, x1);
    omega: angular frequency; pml: absorbing-layer width in grid points on
    all six sides.  Fields are complex128 CUDA tensors of shape (nrhs, n^3)
    (or (n^3,)), x1 fastest.  Face factors are strongly admissible H-matrices
    on quadtree face clusters: leaf (face points per leaf box), rank,
    rank_tol; complex128.
    """

    def __init__(self, c, omega, pml, leaf=16, rank=2, rank_tol=1e-6, restart=40, pml_C=20.0):
        lib = _lib.load()
        if isinstance(c, torch.Tensor):
            c_t = c.detach().to(torch.float64).contiguous()
        else:
            c_t = torch.as_tensor(np.ascontiguousarray(c, dtype=np.float64))
        n = int(c_t.shape[0])
        if c_t.dim() != 3 or tuple(c_t.shape) != (n, n, n):
            raise ValueError("c must be a cubic (n, n, n) array")
        self.n = n
        self._c = c_t
        self._ctx = ctypes.c_void_p()
        _lib.check(lib.hsweep3_setup(ctypes.c_void_p(c_t.data_ptr()), float(omega), int(pml), n,
                                     ctypes.byref(self._ctx)))
        o = _lib.default_opts()
        o.leaf, o.rank, o.rank_tol = int(leaf), int(rank), float(rank_tol)
        o.restart, o.pml_C = int(restart), float(pml_C)
        o.precision = _lib.C128
        o.admissibility = _lib.ADMISSIBILITY["strong"]
        _lib.check(lib.hsweep3_set_opts(self._ctx, ctypes.byref(o)))
        self.factored = False

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            _lib.load().hsweep3_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fields(self, x):
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.complex128:
            raise TypeError("fields must be complex128 CUDA tensors")
        single = x.dim() == 1
        x2 = x.reshape(1, -1) if single else x.reshape(x.shape[0], -1)
        if x2.shape[1] != self.n ** 3:
            raise ValueError(f"each field must have n^3 = {self.n ** 3} entries")
        return x2.contiguous(), single

    def plan_info(self):
        lev, fb = ctypes.c_int(), ctypes.c_size_t()
        _lib.check(_lib.load().hsweep3_plan_info(self._ctx, ctypes.byref(lev), ctypes.byref(fb)))
        return {"levels": lev.value, "factor_bytes": fb.value}

    def factor(self, stream=None):
        _lib.check(_lib.load().hsweep3_factor(self._ctx, _stream_ptr(stream)))
        self.factored = True
        return self

    def apply(self, f, stream=None):
        """u = M f (one face-by-face sweep)."""
        f2, single = self._fields(f)
        u = torch.empty_like(f2)
        _lib.check(_lib.load().hsweep3_apply(self._ctx, ctypes.c_void_p(f2.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                             f2.shape[0], _stream_ptr(stream)))
        return u[0] if single else u

    def stencil(self, x, stream=None):
        """y = A x with the FP64 7-point operator."""
        x2, single = self._fields(x)
        y = torch.empty_like(x2)
        _lib.check(_lib.load().hsweep3_stencil(self._ctx, ctypes.c_void_p(x2.data_ptr()),
                                               ctypes.c_void_p(y.data_ptr()), x2.shape[0], _stream_ptr(stream)))
        return y[0] if single else y

    def solve(self, f, tol=1e-6, maxit=200, stream=None):
        """Flexible GMRES; returns (u, iterations, relative residuals)."""
        f2, single = self._fields(f)
        k = f2.shape[0]
        u = torch.empty_like(f2)
        its = (ctypes.c_int * k)()
        res = (ctypes.c_double * k)()
        _lib.check(_lib.load().hsweep3_solve(self._ctx, ctypes.c_void_p(f2.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                             k, float(tol), int(maxit), its, res, _stream_ptr(stream)))
        if single:
            return u[0], its[0], res[0]
        return u, list(its), list(res)


def factor_batch(solvers, stream=None):
    arr = (ctypes.c_void_p * len(solvers))(*[s._ctx.value for s in solvers])
    _lib.check(_lib.load().hsweep_factor_batch(arr, len(solvers), _stream_ptr(stream)))
    for s in solvers:
        s.factored = True


def solve_batch(solvers, fs, tol=1e-6, maxit=200, stream=None):
    """One right-hand side per solver; returns (list of u, iterations, residuals)."""
    k = len(solvers)
    f2 = [_as_fields(f, s.n)[0] for f, s in zip(fs, solvers)]
    us = [torch.empty_like(f) for f in f2]
    arr = (ctypes.c_void_p * k)(*[s._ctx.value for s in solvers])
    fa = (ctypes.c_void_p * k)(*[f.data_ptr() for f in f2])
    ua = (ctypes.c_void_p * k)(*[u.data_ptr() for u in us])
    its = (ctypes.c_int * k)()
    res = (ctypes.c_double * k)()
    _lib.check(_lib.load().hsweep_solve_batch(arr, k, fa, ua, float(tol), int(maxit), its, res,
                                              _stream_ptr(stream)))
    return [u[0] for u in us], list(its), list(res)


class _HelmholtzSolve(torch.autograd.Function):
    """u = A(c)^{-1} f with gradients through the adjoint sweep.

    A(c) = A(c)^t, so the adjoint field of a real loss L with
    g = dL/dRe(u) + i dL/dIm(u) is mu = A^{-1} conj(g), obtained with the
    same factorization; dL/dc = sum_k Re(mu_k u_k 2 omega^2/((s1 s2) c^3))
    and dL/df = conj(mu).
    """

    @staticmethod
    def forward(ctx, c, f, omega, pml, tol, opts):
        solver = Solver(c.detach(), omega, pml, **opts).factor()
        u, its, res = solver.solve(f.detach(), tol=tol)
        ctx.solver = solver
        ctx.tol = tol
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        solver = ctx.solver
        g = grad_u.resolve_conj().contiguous().to(torch.complex128)
        mu, grad_f, _, _ = solver.solve_adjoint(g, tol=ctx.tol, want_grad_f=bool(ctx.needs_input_grad[1]))
        grad_c = solver.grad_c(u, mu) if ctx.needs_input_grad[0] else None
        return grad_c, grad_f, None, None, None, None


def helmholtz_solve(c, f, omega, pml, tol=1e-10, **opts):
    """Differentiable solve: c (n, n) float64 CUDA tensor, f complex128 (nrhs, n*n)."""
    return _HelmholtzSolve.apply(c, f, float(omega), int(pml), float(tol), opts)
