"""Plain FP64 CPU oracle for the 2D PML Helmholtz sweeping method.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite,
the package smoke check and the CPU-baseline leg of the benchmark may
import it; the GPU library never calls it, and it shares no code with the
GPU library (only the seeded input generators in `workloads` serve both).

Contents, each following a passage of Engquist & Ying, "Sweeping
preconditioner for the Helmholtz equation: hierarchical matrix
representation" (2010):

* pml        -- PML profile sigma(t) and stretching s(t)   (Sec. 2.1, eq. sigma)
* assemble   -- 5-point symmetric PML operator A          (Sec. 2.1, eq. helmd)
* direct     -- u = A^{-1} f by sparse / banded / dense LU (plain definition)
* sweep      -- exact sweeping factorization and solve     (Sec. 2.1, Algs. 2.1-2.2)
* hmatrix    -- weakly admissible H-matrix algebra, the approximate
                factorization and sweep                   (Sec. 2.3-2.4, Algs. 2.3-2.4)
* strong     -- strongly admissible H-matrices with randomized SVD for
                F = H . H, the factorization and sweep in that format
                                                          (Sec. 2.3 strongly admissible case, Algs. 2.3-2.4)
* threed     -- the 3D method: 7-point PML operator, separable closed form,
                exact face-by-face sweep, strongly admissible face
                H-matrices on a quadtree                  (Sec. 4)
* gmres      -- (flexible) GMRES in FP64                   (Sec. 2.4, preconditioned solve)
* fastdiag   -- separable closed form for constant c       (textbook fast diagonalization)
* hankel     -- free-space Green's function reference      (Sec. 2.2, Hankel kernel)
* gradient   -- receiver misfit, adjoint gradient, finite differences
"""
from . import pml, assemble, direct, sweep, gmres, fastdiag, hankel, gradient, hmatrix, strong, threed  # noqa: F401
