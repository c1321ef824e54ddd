"""Host logic of the C-ABI checked on the CPU: the library's host code is
compiled with g++ against a host-memory stand-in of the HIP runtime, and
every kernel launch is replaced by a check that the device ranges it would
touch lie inside live allocations (tests/hostcheck).  The build uses the
address and undefined-behaviour sanitizers.  This caught a work buffer sized
with sizeof of a shadowing bool instead of the element type.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HC = os.path.join(ROOT, "tests", "hostcheck")
EMU = os.path.join(ROOT, "tests", "emucheck")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_launch_ranges_of_batched_and_single_solves(tmp_path):
    exe = str(tmp_path / "hostcheck")
    csrc = os.path.join(ROOT, "paper_1007_4290_amd", "csrc")
    cmd = ["g++", "-std=c++17", "-O0", "-g", "-fsanitize=address,undefined", "-I", EMU, "-I", HC,
           "-I", os.path.join(ROOT, "include"), "-I", csrc,
           "-x", "c++", os.path.join(csrc, "api.hip"), os.path.join(csrc, "strong.hip"), "-x", "none",
           os.path.join(HC, "fake_runtime.cpp"), os.path.join(HC, "stubs.cpp"), os.path.join(EMU, "emu_state.cpp"),
           os.path.join(HC, "main.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and "HOSTCHECK OK" in run.stdout, run.stdout[-2000:] + run.stderr[-2000:]
