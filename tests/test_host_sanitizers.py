"""The host table builder (csrc/bk_tables.cpp: rings, exact N_tri, kept
combinations, bins, model prediction, contraction work items and groups)
built with AddressSanitizer and UndefinedBehaviorSanitizer and run over a
spread of grids, binnings, multipole sets and work-item shapes: no invalid
memory access, leak or undefined behaviour.  Host code only (g++); no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_14513_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "host", "tables_driver.cpp")


@pytest.mark.timeout(600)
def test_table_builder_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "tables_driver")
    build = subprocess.run(
        ["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", CSRC, DRIVER,
         os.path.join(CSRC, "bk_tables.cpp"), "-o", exe, "-lpthread"],
        capture_output=True, text=True)
    if build.returncode != 0 and "asan" in (build.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=500)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr, run.stderr[-4000:]
    assert run.stdout.count(" ok ") == 9, run.stdout
