"""The small dense factorizations of the strongly admissible H-arithmetic
(k_dense.hip: thin QR, one-sided Jacobi SVD, Gauss-Jordan inverse, and the
fused recompression of a sum of two low-rank factorizations), one
wavefront of 64 lanes per matrix, run on the CPU: the kernels are compiled
with g++ against a stand-in of the HIP runtime that runs each lane as a
thread with a real barrier and real shuffles (tests/wavecheck), under the
address and undefined-behaviour sanitizers, with device allocations
starting as NaN bytes.

Each result is checked against what defines it, with numpy for reference
values: Q R = A with Q orthonormal and R upper triangular; A V with V unitary
and mutually orthogonal columns whose norms are A's singular values, the
permutation sorting them, the kept count as specified; A X = I; the
recompression's product equal to the truncated SVD of the sum; the
leaf-block products of an H-matrix product equal to the dense products.  Working sets
below and above the 60 KiB the kernels stage in shared memory are both
covered.  The shapes
cover one and several passes of the column and pair loops, more columns than
rows, zero columns (the zero-padded factor widths), odd and even column
counts and a singular leaf.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1007_4290_amd", "csrc")


@pytest.fixture(scope="module")
def wave(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("wave") / "wave")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-pthread",
           "-I", os.path.join(ROOT, "tests", "wavecheck"), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-x", "c++", os.path.join(CSRC, "k_dense.hip"), "-x", "none",
           os.path.join(ROOT, "tests", "hostcheck", "fake_runtime.cpp"),
           os.path.join(ROOT, "tests", "wavecheck", "main.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, tmp_path, op, A, rows, cols, rmax=0, tol=0.0):
    lda = A.shape[0]
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as fp:
        fp.write(struct.pack("5i", op, rows, cols, lda, rmax))
        fp.write(struct.pack("d", tol))
        fp.write(np.asfortranarray(A, dtype=np.complex128).tobytes(order="F"))
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    return open(fout, "rb").read()


def _mat(buf, off, rows, cols):
    n = rows * cols
    M = np.frombuffer(buf, dtype=np.complex128, count=n, offset=off).reshape(cols, rows).T
    return M, off + 16 * n


def _rand(rng, m, n):
    return rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))


# working sets below and above the 60 KiB that the kernels stage in shared memory
QR_CASES = [(1, 1), (5, 3), (3, 5), (64, 10), (130, 7), (20, 70), (33, 33), (200, 2), (300, 10)]


@pytest.mark.parametrize("p, k", QR_CASES)
def test_qr(wave, tmp_path, p, k):
    rng = np.random.default_rng(100 + p + 7 * k)
    A = _rand(rng, p + 3, k)                      # leading dimension p + 3
    if k >= 4:
        A[:, 1] = 0.0                             # a zero column
        A[:, 3] = 2.0 * A[:, 2]                   # a dependent one
    out = _run(wave, tmp_path, 0, A, p, k)
    kk = min(p, k)
    Q, off = _mat(out, 0, p, kk)
    R, off = _mat(out, off, kk, k)
    Qc, _ = _mat(out, off, p, kk)
    assert np.array_equal(Qc, Q.conj())
    a = A[:p]
    assert np.allclose(Q.conj().T @ Q, np.eye(kk), atol=1e-13)
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.linalg.norm(Q @ R - a) <= 1e-13 * max(np.linalg.norm(a), 1.0)


SVD_CASES = [(1, 1), (4, 2), (6, 9), (20, 11), (12, 12), (3, 40), (10, 130), (70, 5)]


@pytest.mark.parametrize("a, b", SVD_CASES)
def test_svd(wave, tmp_path, a, b):
    rng = np.random.default_rng(200 + a + 3 * b)
    A = _rand(rng, a + 2, b)
    if b >= 3:
        A[:, b - 1] = 0.0                         # a zero column
    tol, rmax = 1e-6, max(1, min(a, b) - 1)
    out = _run(wave, tmp_path, 1, A, a, b, rmax=rmax, tol=tol)
    AV, off = _mat(out, 0, a + 2, b)
    V, off = _mat(out, off, b, b)
    sig = np.frombuffer(out, dtype=np.float64, count=b, offset=off)
    off += 8 * b
    perm = np.frombuffer(out, dtype=np.int32, count=b, offset=off)
    off += 4 * b
    rank = struct.unpack_from("i", out, off)[0]
    a0 = A[:a]
    assert np.allclose(AV[a:], A[a:]), "rows past the matrix were written"
    assert np.allclose(V.conj().T @ V, np.eye(b), atol=1e-12)
    assert np.linalg.norm(a0 @ V - AV[:a]) <= 1e-12 * np.linalg.norm(a0)
    G = AV[:a].conj().T @ AV[:a]
    nrm = np.sqrt(np.abs(np.diag(G)))
    off_diag = np.abs(G - np.diag(np.diag(G)))
    assert np.all(off_diag <= 1e-12 * np.outer(nrm, nrm) + 1e-13 * nrm.max() ** 2)
    assert np.allclose(sig, nrm, rtol=1e-13, atol=1e-14 * nrm.max())
    assert sorted(perm.tolist()) == list(range(b))
    assert np.all(np.diff(sig[perm]) <= 0.0)
    ref = np.linalg.svd(a0, compute_uv=False)
    assert np.allclose(sig[perm][:len(ref)], ref, rtol=1e-11, atol=1e-13 * ref[0])
    assert np.all(sig[perm][len(ref):] <= 1e-13 * ref[0])
    want = min(int(np.sum(sig > tol * sig.max())), rmax)
    assert rank == want


@pytest.mark.parametrize("m", [1, 2, 7, 16, 33, 40, 50])
def test_inverse(wave, tmp_path, m):
    rng = np.random.default_rng(300 + m)
    A = _rand(rng, m + 1, m)
    if m >= 2:
        A[0, 0] = 0.0                             # needs a row exchange
    out = _run(wave, tmp_path, 2, A, m, m)
    X, off = _mat(out, 0, m, m)
    st = struct.unpack_from("i", out, off)[0]
    assert st == 0
    assert np.linalg.norm(A[:m] @ X - np.eye(m)) <= 1e-11 * np.linalg.cond(A[:m])


def test_inverse_of_a_singular_leaf_sets_the_status(wave, tmp_path):
    rng = np.random.default_rng(7)
    A = _rand(rng, 6, 6)
    A[:, 4] = 0.0
    out = _run(wave, tmp_path, 2, A, 6, 6)
    assert struct.unpack_from("i", out, 16 * 36)[0] == 1


REC_CASES = [(12, 9, 2, 3, 1e-6), (40, 33, 4, 4, 1e-6), (70, 66, 8, 10, 1e-10), (5, 30, 3, 4, 0.0),
             (16, 16, 0, 5, 1e-6), (24, 20, 6, 0, 1e-6)]


def _recompress(exe, tmp_path, cases, rmax):
    """Run the cases (m, q, k1, k2, tol: one tol for all) as one batched launch;
    returns [(inputs, ou, ov)]."""
    tol = cases[0][4]
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    jobs = []
    with open(fin, "wb") as fp:
        fp.write(struct.pack("5i", 3, len(cases), rmax, 0, rmax))
        fp.write(struct.pack("d", tol))
        for t, (m, q, k1, k2, _) in enumerate(cases):
            rng = np.random.default_rng(400 + m + q + k1 + k2 + t)
            alpha = 0.7 - 0.4j
            # factors of decaying weight, so that the truncation is well defined
            au, av = _rand(rng, m, k1) * 2.0 ** -np.arange(k1), _rand(rng, q, k1)
            U, V = _rand(rng, m, k2) * 3.0 ** -np.arange(k2), _rand(rng, q, k2)
            fp.write(struct.pack("5i", 0, m, q, k1, k2))
            fp.write(struct.pack("2d", alpha.real, alpha.imag))
            for M in (au, av, U, V):
                fp.write(np.asfortranarray(M, dtype=np.complex128).tobytes(order="F"))
            jobs.append((m, q, k1, k2, alpha, au, av, U, V))
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    out = open(fout, "rb").read()
    res, off = [], 0
    for (m, q, k1, k2, alpha, au, av, U, V) in jobs:
        width = min(m, q, k1 + k2, rmax)
        ou, off = _mat(out, off, m, width)
        ov, off = _mat(out, off, q, width)
        res.append(((alpha, au, av, U, V), ou, ov))
    return res


def _check_truncation(inputs, ou, ov, tol, rmax):
    alpha, au, av, U, V = inputs
    full = np.hstack([au, alpha * U]) @ np.hstack([av, V]).T
    Uf, s, Vh = np.linalg.svd(full)
    keep = min(int(np.sum(s > (tol * s[0] if tol > 0 else 0.0))), rmax)
    best = (Uf[:, :keep] * s[:keep]) @ Vh[:keep]
    assert np.linalg.norm(ou @ ov.T - best) <= 1e-12 * s[0]
    # columns past the kept rank are zero
    assert np.all(ou[:, keep:] == 0) and np.all(ov[:, keep:] == 0)


@pytest.mark.parametrize("case", REC_CASES)
def test_recompression(wave, tmp_path, case):
    """One recompression gives the truncated SVD of [au, alpha U] [av, V]^t:
    the kept rank's leading singular triplets, zero columns past it."""
    rmax = 8 if case[2] + case[3] >= 16 else max(2, case[2])
    (inputs, ou, ov), = _recompress(wave, tmp_path, [case], rmax)
    _check_truncation(inputs, ou, ov, case[4], rmax)


def test_recompression_batch(wave, tmp_path):
    """Thirty-four jobs in one call (two launches of up to 32 workgroups), with
    working sets in and beyond the 60 KiB of shared memory side by side."""
    cases = [REC_CASES[t % 2][:4] + (1e-6,) for t in range(33)] + [REC_CASES[2][:4] + (1e-6,)]
    for (inputs, ou, ov), c in zip(_recompress(wave, tmp_path, cases, 6), cases):
        _check_truncation(inputs, ou, ov, 1e-6, 6)


@pytest.mark.parametrize("assign", [0, 1])
@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("ncol, rank", [(1, 2), (3, 6), (40, 120)])
def test_leaf_block_products(wave, tmp_path, assign, trans, ncol, rank):
    """Y += alpha op(block) X (Y = ... when assigning) over dense and
    factorized leaf blocks whose output rows are disjoint (one class of a
    product over an H-matrix), for the blocks and their transposes, with a
    block of cleared rows; the largest case keeps its r x ncol temporaries in
    device memory instead of shared memory."""
    rng = np.random.default_rng(500 + 7 * trans + ncol + 3 * assign)
    # output row ranges [0,8), [8,24), [24,30), [40,56), [60,61), cleared [30,40); input rows anywhere
    spec = [(0, 8, 12, 0, 0), (1, 16, 10, 8, 20), (0, 6, 6, 24, 3), (1, 16, 16, 40, 0), (0, 1, 30, 60, 1),
            (2, 10, 0, 30, 0)]
    rows_x, rows_y = 70, 64
    X = _rand(rng, rows_x, ncol)
    Y = _rand(rng, rows_y, ncol)
    alpha = -0.3 + 1.1j
    ref = Y.copy()
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as fp:
        fp.write(struct.pack("5i", 4, len(spec), trans + 2 * assign, ncol, 0))
        fp.write(struct.pack("d", 0.0))
        fp.write(struct.pack("2i", rows_x, rows_y))
        fp.write(struct.pack("2d", alpha.real, alpha.imag))
        for M in (X, Y):
            fp.write(np.asfortranarray(M).tobytes(order="F"))
        for kind, out, inn, yo, xo in spec:
            if kind == 2:
                fp.write(struct.pack("6i", 2, out, out, 0, yo, 0))
                ref[yo:yo + out] = 0.0
                continue
            # the block is m x q; op(block) maps `inn` input rows to `out` output rows
            m, q = (inn, out) if trans else (out, inn)
            r = rank if kind else 0
            fp.write(struct.pack("6i", kind, m, q, r, yo, xo))
            if kind == 0:
                D = _rand(rng, m, q)
                blk = D
                fp.write(np.asfortranarray(D).tobytes(order="F"))
            else:
                U, V = _rand(rng, m, r), _rand(rng, q, r)
                blk = U @ V.T
                fp.write(np.asfortranarray(U).tobytes(order="F"))
                fp.write(np.asfortranarray(V).tobytes(order="F"))
            op = blk.T if trans else blk
            ref[yo:yo + out] = (0.0 if assign else ref[yo:yo + out]) + alpha * (op @ X[xo:xo + inn])
    r = subprocess.run([wave, fin, fout], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    out = np.frombuffer(open(fout, "rb").read(), dtype=np.complex128).reshape(ncol, rows_y).T
    assert np.linalg.norm(out - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("a, b", [(16, 10), (30, 12)])
def test_svd_with_a_cut_keeps_the_leading_triplets(wave, tmp_path, a, b):
    """Singular values graded from 1 down to 1e-13 and a cut at 1e-6: the
    kept triplets match numpy, the kept count is the number above the cut,
    and the columns past it stay below the cut."""
    rng = np.random.default_rng(600 + a + b)
    Uq, _ = np.linalg.qr(_rand(rng, a, b))
    Vq, _ = np.linalg.qr(_rand(rng, b, b))
    sv = 10.0 ** -np.linspace(0, 13, b)
    A = (Uq * sv) @ Vq.conj().T
    tol, rmax = 1e-6, b
    out = _run(wave, tmp_path, 1, A, a, b, rmax=rmax, tol=tol)
    AV, off = _mat(out, 0, a, b)
    V, off = _mat(out, off, b, b)
    sig = np.frombuffer(out, dtype=np.float64, count=b, offset=off)
    off += 8 * b
    perm = np.frombuffer(out, dtype=np.int32, count=b, offset=off)
    off += 4 * b
    rank = struct.unpack_from("i", out, off)[0]
    keep = int(np.sum(sv > tol * sv[0]))
    assert rank == keep
    assert np.allclose(V.conj().T @ V, np.eye(b), atol=1e-12)
    assert np.linalg.norm(A @ V - AV) <= 1e-12 * np.linalg.norm(A)
    assert np.allclose(sig[perm][:keep], sv[:keep], rtol=1e-10)
    assert np.all(sig[perm][keep:] < tol * sv[0])
    # the kept left directions are orthonormal and match the truncated SVD
    Ur = AV[:, perm[:keep]] / sig[perm[:keep]]
    assert np.allclose(Ur.conj().T @ Ur, np.eye(keep), atol=1e-10)
    best = (Uq[:, :keep] * sv[:keep]) @ Vq[:, :keep].conj().T
    approx = AV[:, perm[:keep]] @ V[:, perm[:keep]].conj().T
    assert np.linalg.norm(approx - best) <= 1e-10


def test_dense_block_jobs(wave, tmp_path):
    """The dense kinds of a block-job batch, side by side with a
    recompression in one launch: a sum, a low-rank update, a row-and-column
    scaling and a copy."""
    rng = np.random.default_rng(700)
    alpha = 0.4 + 0.9j
    m, q, k2 = 13, 9, 3
    A, Bm, O = _rand(rng, m, q), _rand(rng, m, q), _rand(rng, m, q)
    U, V = _rand(rng, m, k2), _rand(rng, q, k2)
    dl, dr = _rand(rng, m, 1)[:, 0], _rand(rng, q, 1)[:, 0]
    # (kind, data arrays in file order, expected)
    jobs = [(1, [A, Bm, O], A + alpha * Bm),
            (2, [A, U, V, O], O + alpha * U @ V.T),
            (3, [A, dl, dr, O], dl[:, None] * A * dr[None, :]),
            (4, [A, O], A)]
    rec = REC_CASES[0]
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    rec_rng = np.random.default_rng(9)
    with open(fin, "wb") as fp:
        fp.write(struct.pack("5i", 3, len(jobs) + 1, 2, 0, 2))
        fp.write(struct.pack("d", 1e-6))
        for kind, arrs, _ in jobs:
            fp.write(struct.pack("5i", kind, m, q, 0, k2 if kind == 2 else 0))
            fp.write(struct.pack("2d", alpha.real, alpha.imag))
            for M in arrs:
                fp.write(np.asfortranarray(np.asarray(M, dtype=np.complex128)).tobytes(order="F"))
        mm, qq, k1r, k2r = rec[:4]
        au, av = _rand(rec_rng, mm, k1r), _rand(rec_rng, qq, k1r)
        Ur, Vr = _rand(rec_rng, mm, k2r), _rand(rec_rng, qq, k2r)
        fp.write(struct.pack("5i", 0, mm, qq, k1r, k2r))
        fp.write(struct.pack("2d", alpha.real, alpha.imag))
        for M in (au, av, Ur, Vr):
            fp.write(np.asfortranarray(M).tobytes(order="F"))
    r = subprocess.run([wave, fin, fout], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    out = open(fout, "rb").read()
    off = 0
    for kind, _, want in jobs:
        got, off = _mat(out, off, m, q)
        assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want), kind
    width = min(mm, qq, k1r + k2r, 2)
    ou, off = _mat(out, off, mm, width)
    ov, off = _mat(out, off, qq, width)
    _check_truncation((alpha, au, av, Ur, Vr), ou, ov, 1e-6, 2)


def test_randomized_svd_tails(wave, tmp_path):
    """Three randomized-SVD tails in one launch (one staged in shared memory,
    one too large for it, one square): Uo Vo^t is the truncated SVD of Q M^t,
    with Q an orthonormal sample basis, rank capped at rmax and cut at tol."""
    rng = np.random.default_rng(800)
    rmax, tol = 3, 1e-6
    cases = [(24, 20, 10), (200, 420, 10), (12, 10, 10)]
    data = []
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as fp:
        fp.write(struct.pack("5i", 5, len(cases), 0, 0, rmax))
        fp.write(struct.pack("d", tol))
        for m, q, ell in cases:
            Q, _ = np.linalg.qr(_rand(rng, m, ell))
            # a projected block with a decaying spectrum
            M = (_rand(rng, q, ell) * 4.0 ** -np.arange(ell)) @ np.linalg.qr(_rand(rng, ell, ell))[0]
            fp.write(struct.pack("3i", m, q, ell))
            fp.write(np.asfortranarray(Q).tobytes(order="F"))
            fp.write(np.asfortranarray(M).tobytes(order="F"))
            data.append((Q, M))
    r = subprocess.run([wave, fin, fout], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    out = open(fout, "rb").read()
    off = 0
    for (m, q, ell), (Q, M) in zip(cases, data):
        w = min(ell, rmax)
        Uo, off = _mat(out, off, m, w)
        Vo, off = _mat(out, off, q, w)
        full = Q @ M.T
        Uf, sv, Vh = np.linalg.svd(full, full_matrices=False)
        keep = min(int(np.sum(sv > tol * sv[0])), rmax)
        best = (Uf[:, :keep] * sv[:keep]) @ Vh[:keep]
        assert np.linalg.norm(Uo @ Vo.T - best) <= 1e-12 * sv[0]
