"""The kernels' exact-arithmetic header (fp64 quotients, modular multiply and inverse, the
Eq. 4-5 solver in offset form, the per-prime driver loop and the three-gap stepping rule),
compiled for the host with g++ and checked against brute force and 128-bit integers."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_arith_header_against_brute_force(tmp_path, seed):
    exe = str(tmp_path / "arith_check")
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(ROOT, "tests", "arith_host_check.cpp"),
                    "-o", exe], check=True)
    out = subprocess.run([exe, str(seed)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "OK" in out.stdout
