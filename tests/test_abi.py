"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and validates arguments on the host before any device work."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_1007_4290_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsweep.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hsweep3?_\w+)\s*\(", txt)))


def test_header_declares_the_binding_symbols():
    assert _declared() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_options():
    o = _lib.default_opts()
    assert (o.leaf, o.rank, o.precision, o.dense) == (16, 8, _lib.C128, 0)
    assert o.rank_tol == pytest.approx(1e-6)
    assert o.pml_C == pytest.approx(20.0)
    assert o.admissibility == _lib.ADMISSIBILITY["weak"]
    assert tuple(o.pml_sides) == (-1, -1, -1, -1)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_binding_options_struct_matches_the_header(tmp_path):
    # the ctypes mirror of hsweep_opts has the C layout: size and every offset
    src = tmp_path / "opts.c"
    fields = [f[0] for f in _lib.Opts._fields_]
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hsweep.h"\nint main(void) {\n'
                   '  printf("%zu\\n", sizeof(hsweep_opts));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(hsweep_opts, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "opts"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(_lib.Opts)
    assert vals[1:] == [getattr(_lib.Opts, f).offset for f in fields]


def _setup(c, omega, pml, n):
    lib = _lib.load()
    ctx = ctypes.c_void_p()
    arr = np.ascontiguousarray(c, dtype=np.float64)
    rc = lib.hsweep_setup(arr.ctypes.data_as(ctypes.c_void_p), omega, pml, n, ctypes.byref(ctx))
    return rc, ctx


@pytest.mark.parametrize("n,omega,pml,fill,code", [
    (2, 10.0, 0, 1.0, _lib.EINVAL),        # n < 3
    (16, 0.0, 2, 1.0, _lib.EINVAL),        # omega <= 0
    (16, float("inf"), 2, 1.0, _lib.EINVAL),
    (16, 10.0, -1, 1.0, _lib.EINVAL),      # pml < 0
    (16, 10.0, 8, 1.0, _lib.EINVAL),       # 2 pml >= n
    (16, 10.0, 2, 0.0, _lib.EINVAL),       # c <= 0
    (16, 10.0, 2, float("nan"), _lib.EINVAL),
])
def test_setup_rejects_invalid_arguments(n, omega, pml, fill, code):
    c = np.full((max(n, 1), max(n, 1)), fill)
    rc, ctx = _setup(c, omega, pml, n)
    assert rc == code
    assert ctx.value is None
    assert len(_lib.load().hsweep_last_error()) > 0


def test_setup_rejects_one_bad_velocity_value():
    c = np.ones((16, 16))
    c[5, 7] = -1.0
    rc, _ = _setup(c, 10.0, 2, 16)
    assert rc == _lib.EINVAL


def test_null_arguments_are_rejected():
    lib = _lib.load()
    assert lib.hsweep_setup(None, 1.0, 0, 8, ctypes.byref(ctypes.c_void_p())) == _lib.EINVAL
    assert lib.hsweep_factor(None, None) == _lib.EINVAL
    assert lib.hsweep_apply(None, None, None, 1, None) == _lib.EINVAL
    assert lib.hsweep_solve(None, None, None, 1, 1e-6, 10, None, None, None) == _lib.EINVAL
    assert lib.hsweep_set_opts(None, None) == _lib.EINVAL
    assert lib.hsweep_timings(None, None, 0) == _lib.EINVAL
    assert lib.hsweep_factor_profile(None, None, None, 3) == _lib.EINVAL
    assert lib.hsweep_solve_adjoint(None, None, None, None, 1, 1e-6, 10, None, None, None) == _lib.EINVAL
    assert lib.hsweep_workspace_bytes(None, 1, None, None) == _lib.EINVAL
    lib.hsweep_destroy(None)


def test_valid_setup_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, ctx = _setup(np.ones((15, 15)), 20.0, 2, 15)
    assert rc == _lib.EDEVICE
    assert ctx.value is None
