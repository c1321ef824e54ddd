"""The library's 3D path (Sec. 4: the 7-point operator and the face-by-face
sweep with strongly admissible face H-matrices on quadtree clusters) run on
the CPU through the kernel emulation of tests/emucheck (api3.hip, the
coefficient kernels and strong.hip compiled with g++ under the address and
undefined-behaviour sanitizers, device allocations starting as NaN bytes),
against the oracle's 3D operator and sparse LU:

* the FP64 operator equals the oracle's;
* untruncated face factors make the sweep the exact inverse;
* rank-2 face factors at tolerance 1e-6 precondition FP64 GMRES to the
  solution in as many iterations as the oracle's (7 at n = 15).
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import threed as T3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emucheck")
HC = os.path.join(ROOT, "tests", "hostcheck")
CSRC = os.path.join(ROOT, "paper_1007_4290_amd", "csrc")


@pytest.fixture(scope="module")
def emu3(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("emu3") / "emu3")
    srcs = [os.path.join(CSRC, f) for f in ("api.hip", "api3.hip", "k_coeff.hip", "k_coeff3.hip", "strong.hip")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-I", EMU, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "c++", *srcs, "-x", "none",
           os.path.join(HC, "fake_runtime.cpp"), os.path.join(EMU, "emu_state.cpp"),
           os.path.join(EMU, "cpu_kernels.cpp"), os.path.join(EMU, "dense_cpu.cpp"), os.path.join(EMU, "main3.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, tmp_path, c, omega, pml, F, leaf, rank, tol, mode, gtol=1e-10, maxit=50):
    n = c.shape[0]
    nrhs = F.shape[0]
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as fp:
        fp.write(struct.pack("7i", n, pml, leaf, rank, nrhs, mode, maxit))
        fp.write(struct.pack("3d", omega, tol, gtol))
        fp.write(np.ascontiguousarray(c, dtype=np.float64).tobytes())
        fp.write(np.ascontiguousarray(F, dtype=np.complex128).tobytes())
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=900,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    b = open(fout, "rb").read()
    rc, levels = struct.unpack_from("2i", b, 0)
    o = 8
    its = np.frombuffer(b, np.int32, nrhs, o)
    o += 4 * nrhs
    res = np.frombuffer(b, np.float64, nrhs, o)
    o += 8 * nrhs
    fbytes, = struct.unpack_from("Q", b, o)
    o += 8
    u = np.frombuffer(b, np.complex128, nrhs * n ** 3, o).reshape(nrhs, n ** 3)
    return dict(rc=rc, levels=levels, its=its, res=res, fbytes=fbytes, u=u)


def _close(u, ue, tol):
    assert np.abs(u - ue).max() <= tol * np.abs(ue).max()
    assert np.linalg.norm(u - ue) <= tol * np.linalg.norm(ue)


def _medium(n, seed):
    return 1 + 0.3 * np.random.default_rng(seed).random((n, n, n))


def _centre_source(n):
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    s = 1.5 * h
    g = np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5
    return g.ravel().astype(complex)


def test_operator_equals_the_oracle(emu3, tmp_path):
    n, om, pml = 7, 2 * np.pi * 1.5, 2
    c = _medium(n, 1)
    F = np.random.default_rng(2).standard_normal((2, n ** 3)) + 1j * np.random.default_rng(3).standard_normal((2, n ** 3))
    out = _run(emu3, tmp_path, c, om, pml, F, 4, 16, 0.0, mode=2)
    _close(out["u"], T3.apply(T3.stencil(c, om, pml), F), 1e-13)


@pytest.mark.parametrize("n", [7, 8])
def test_untruncated_face_factors_are_the_exact_inverse(emu3, tmp_path, n):
    om, pml = 2 * np.pi * 1.5, 2
    c = _medium(n, n)
    rng = np.random.default_rng(5)
    F = rng.standard_normal((2, n ** 3)) + 1j * rng.standard_normal((2, n ** 3))
    out = _run(emu3, tmp_path, c, om, pml, F, 4, 64, 0.0, mode=0)
    assert out["rc"] == 0 and out["levels"] == 4 and out["fbytes"] > 0
    Ue = spla.spsolve(T3.matrix(T3.stencil(c, om, pml)).tocsc(), F.T).T
    for k in range(2):
        _close(out["u"][k], Ue[k], 1e-10)


def test_rank_two_face_factors_precondition_gmres_to_the_solution(emu3, tmp_path):
    n, om, pml = 15, 2 * np.pi * 2, 3
    c = _medium(n, 13)
    f = _centre_source(n).reshape(1, -1)
    out = _run(emu3, tmp_path, c, om, pml, f, 16, 2, 1e-6, mode=1)
    assert out["rc"] == 0 and out["res"][0] <= 1e-10 and out["its"][0] <= 10
    ue = spla.spsolve(T3.matrix(T3.stencil(c, om, pml)).tocsc(), f[0])
    _close(out["u"][0], ue, 1e-8)
