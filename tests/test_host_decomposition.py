"""The contraction's work decomposition, checked on the host: every kept
combination is summed in a cell of its own that stages three real sides on
the planes (a, b, a + b) of a canonical plane triple, on a grid that cannot
alias its rings' closures (m > U_A + U_B + U_C and m > 2 max U, U from the
rings' lattice modes); groups keep to their slot and item limits and grid
sides sit back to back in D.  The checker is tests/host/decomposition_check.cpp,
compiled with g++ against the table builder.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_14513_amd", "csrc")


@pytest.mark.timeout(600)
def test_work_decomposition_is_exact_and_within_limits(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "decomposition_check")
    build = subprocess.run(
        ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC,
         os.path.join(ROOT, "tests", "host", "decomposition_check.cpp"), os.path.join(CSRC, "bk_tables.cpp"),
         "-o", exe, "-lpthread"], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=500)
    assert run.returncode == 0, run.stdout[-3000:]
    assert run.stdout.count(" ok: ") == 8, run.stdout
