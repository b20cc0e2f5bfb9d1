"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host-side code
(no GPU): the C oracle, exercised on thin and odd grids with every boundary
mix, and the systolic launch plan (paper_2502_20610_amd/csrc/plan.cpp), checked
for coverage, topological order, ring-group contiguity and the merged-launch
distance bound.  Built with gcc/g++ here; any sanitizer report aborts the
program (-fno-sanitize-recover), so a clean exit is the pass."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _have(tool):
    return shutil.which(tool) is not None


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    if "does not come first in initial library list" in r.stderr:
        pytest.skip("another preloaded library precedes the AddressSanitizer runtime here")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(not _have("gcc"), reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.run(["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off"] + SAN +
                   [os.path.join(ROOT, "oracle", "yee_oracle.c"),
                    os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"), "-lm", "-o", exe],
                   check=True)
    assert "passed" in _run(exe)


@pytest.mark.skipif(not _have("g++"), reason="g++ not found")
def test_plan_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    csrc = os.path.join(ROOT, "paper_2502_20610_amd", "csrc")
    subprocess.run(["g++", "-std=c++17"] + SAN + ["-I" + csrc, os.path.join(csrc, "plan.cpp"),
                    os.path.join(ROOT, "tests", "sanitize", "plan_check.cpp"), "-o", exe], check=True)
    assert "plan checks passed" in _run(exe)
