"""The library's strongly admissible path (Sec. 2.3, strongly admissible
case) run on the CPU: api.hip, the coefficient kernels and strong.hip are
compiled with g++ against a host stand-in of the HIP runtime whose launch
calls each kernel once per (block, thread) index (tests/emucheck), under the
address and undefined-behaviour sanitizers, with every device allocation
starting as NaN bytes.  Compared with the oracle's sparse LU solution:

* untruncated strong factors (tolerance 0, rank cap above every block's
  size) make the sweep the exact inverse, also with absorbing-condition
  sides;
* rank-2 factors at tolerance 1e-6 precondition FP64 GMRES to the solution
  in a handful of iterations, in each sweep direction.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from oracle import assemble, direct
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emucheck")
HC = os.path.join(ROOT, "tests", "hostcheck")
CSRC = os.path.join(ROOT, "paper_1007_4290_amd", "csrc")


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("emu") / "emu")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-I", EMU, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-x", "c++", os.path.join(CSRC, "api.hip"), os.path.join(CSRC, "k_coeff.hip"),
           os.path.join(CSRC, "strong.hip"), "-x", "none",
           os.path.join(HC, "fake_runtime.cpp"), os.path.join(EMU, "emu_state.cpp"),
           os.path.join(EMU, "cpu_kernels.cpp"), os.path.join(EMU, "dense_cpu.cpp"), os.path.join(EMU, "main.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, tmp_path, c, omega, pml, F, leaf, rank, tol, direction=0, solve=False, gtol=1e-10, maxit=50,
         sides=(-1, -1, -1, -1)):
    n = c.shape[0]
    nrhs = F.shape[0]
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as fp:
        fp.write(struct.pack("12i", n, pml, leaf, rank, direction, nrhs, int(solve), maxit, *sides))
        fp.write(struct.pack("3d", omega, tol, gtol))
        fp.write(np.ascontiguousarray(c, dtype=np.float64).tobytes())
        fp.write(np.ascontiguousarray(F, dtype=np.complex128).tobytes())
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    b = open(fout, "rb").read()
    rc, n_p, levels = struct.unpack_from("3i", b, 0)
    o = 12
    its = np.frombuffer(b, np.int32, nrhs, o)
    o += 4 * nrhs
    res = np.frombuffer(b, np.float64, nrhs, o)
    o += 8 * nrhs
    fbytes, = struct.unpack_from("Q", b, o)
    o += 8
    u = np.frombuffer(b, np.complex128, nrhs * n * n, o).reshape(nrhs, n * n)
    return dict(rc=rc, n_p=n_p, levels=levels, its=its, res=res, fbytes=fbytes, u=u)


def _close(u, ue, tol):
    scale = np.abs(ue).max()
    assert np.abs(u - ue).max() <= tol * scale
    assert np.linalg.norm(u - ue) <= tol * np.linalg.norm(ue)


@pytest.mark.parametrize("n, leaf, direction, sides", [
    (31, 4, 0, (-1, -1, -1, -1)),
    (31, 4, 1, (-1, -1, -1, -1)),
    (31, 4, 2, (-1, -1, -1, -1)),
    (31, 4, 0, (2, 5, 3, 4)),                    # a different layer width per side
    (37, 4, 0, (2, 5, 3, 4)),                    # and an uneven bisection
    (31, 4, 0, ("abc", 4, 0, "abc")),            # absorbing-condition, layered and Dirichlet sides
])
def test_untruncated_strong_factors_are_the_exact_inverse(emu, tmp_path, n, leaf, direction, sides):
    c = W.random_field_medium(n, 41)
    om = 2 * np.pi * 4
    widths = tuple(0 if v == "abc" else v for v in sides)
    abc = tuple(e for e, v in zip(assemble.EDGES, sides) if v == "abc")
    st = assemble.stencil(c, om, tuple(4 if w == -1 else w for w in widths), abc=abc)
    rng = np.random.default_rng(7)
    F = rng.standard_normal((2, n * n)) + 1j * rng.standard_normal((2, n * n))
    code = tuple(-2 if v == "abc" else v for v in sides)
    out = _run(emu, tmp_path, c, om, 4, F, leaf=leaf, rank=16, tol=0.0, sides=code, direction=direction)
    assert out["rc"] == 0 and out["n_p"] == n and out["fbytes"] > 0
    Ue = direct.solve_sparse(st, F)
    for k in range(2):
        _close(out["u"][k], Ue[k], 1e-10)


@pytest.mark.parametrize("direction", [0, 1, 2])
def test_rank_two_strong_factors_precondition_gmres_to_the_solution(emu, tmp_path, direction):
    n = 63
    c = W.random_field_medium(n, 1)
    om = 2 * np.pi * 8
    f = W.gaussian_source(n, (0.5, 0.5)).reshape(1, -1)
    out = _run(emu, tmp_path, c, om, 12, f, leaf=8, rank=2, tol=1e-6, direction=direction, solve=True)
    assert out["rc"] == 0 and out["res"][0] <= 1e-10
    assert out["its"][0] <= 5
    _close(out["u"][0], direct.solve_sparse(assemble.stencil(c, om, 12), f[0]), 1e-8)


def test_rank_two_strong_factors_two_sources_n127(emu, tmp_path):
    n = 127
    c = W.random_field_medium(n, 43)
    om = 2 * np.pi * 16
    F = np.stack([W.gaussian_source(n, (0.4, 0.6)).ravel(), W.gaussian_source(n, (0.7, 0.3)).ravel()]).astype(complex)
    out = _run(emu, tmp_path, c, om, 12, F, leaf=16, rank=2, tol=1e-6, solve=True)
    assert out["rc"] == 0 and out["levels"] == 3 and max(out["res"]) <= 1e-10 and max(out["its"]) <= 6
    Ue = direct.solve_sparse(assemble.stencil(c, om, 12), F)
    for k in range(2):
        _close(out["u"][k], Ue[k], 1e-8)
