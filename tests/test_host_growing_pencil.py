"""The incremental subspace solve of the Davidson iteration
(sph::GrowingPencil, host code) against the full one (sph::gen_lowest): the
same bits on pencils that grow by one row and column per call, and the full
solve taken whenever nothing certifies that canonical orthogonalisation
keeps every direction.  Builds tests/cpp/growing_pencil_check.cpp with the
library's host numerics (host_linalg.cpp) and runs it on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1703_04789_amd", "csrc")


def test_growing_pencil_matches_the_full_solve(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "growing_pencil_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I" + CSRC, os.path.join(ROOT, "tests", "cpp", "growing_pencil_check.cpp"),
                    os.path.join(CSRC, "host_linalg.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
