"""CPU check of the step kernel's index arithmetic (no GPU): the LDS layout's
regions stay inside the working set and the regions live at the same time
are disjoint, the narrowphase staging and the solver records stay inside a
scene's record block, and the packed key fields hold every body index, over
the scene sizes and capacities the host accepts.  The checker is plain C++
built here with g++ against the kernel's own layout header."""
import os
import shutil
import subprocess

import pytest

from helpers import ROOT

SRC = os.path.join(ROOT, "tests", "native", "index_math.cpp")


def test_kernel_index_math(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "index_math")
    subprocess.run([gxx, "-O1", "-std=c++17", "-Wall", "-Werror", "-o", exe, SRC], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr + r.stdout
    assert "failures: 0" in r.stdout
