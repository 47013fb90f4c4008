"""The header is plain C: a C99 program (tests/c/abi_check.c) compiles
against include/mpcd.h with all warnings as errors, links libmpcd.so and
calls host-only entry points (mpcd_footprint, argument validation), which
give what the Python binding gives."""
import os
import shutil
import subprocess

import pytest

from paper_1801_10187_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_program_uses_the_abi(tmp_path):
    exe = str(tmp_path / "abi_check")
    libdir = os.path.dirname(binding.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "abi_check.c"),
                    "-L", libdir, "-lmpcd", f"-Wl,-rpath,{libdir}", "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    line = [l for l in r.stdout.splitlines() if l.startswith("footprint")][0]
    peak, held = (int(x) for x in line.split()[1:])
    assert (peak, held) == binding.footprint((50, 50, 50), 10**6, nsteps=10, precision=binding.FP32,
                                             tile="4x4x4")
    assert "MPCD_EINVAL" in r.stdout or "bad cell size: 1" in r.stdout
