"""The reduced-basis table of the x pass (csrc/basis.hpp), checked on the host: for random
unit vectors every dependent monomial (power of rhat_z >= 2) equals its combination of the
gathered ones, from the identity rhat_x^2 + rhat_y^2 + rhat_z^2 = 1 (Sec. 3, Eqs. 11 and 13
grids). The header is compiled as plain C++ by a small driver program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_reduced_basis_table(tmp_path):
    gxx = shutil.which("g++") or shutil.which("c++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "basis_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-D__host__=", "-D__device__=",
                    "-I" + os.path.join(ROOT, "paper_1505_05341_amd", "csrc"),
                    os.path.join(ROOT, "tests", "basis_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
