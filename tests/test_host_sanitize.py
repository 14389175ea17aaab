"""The host entry points (exact-predicate Delaunay in 3-D and in the plane,
the Z/2 persistence reduction) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on random sets, lattices whose every
empty-sphere test is a tie, near-degenerate perturbations of them and sets
that must be refused (tests/host_sanitize.cpp).  Host code only: g++ builds
the two host sources with the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_22432_amd", "csrc")


@pytest.mark.timeout(600)
def test_host_code_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "host_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host_sanitize.cpp"), os.path.join(CSRC, "delaunay.cpp"),
           os.path.join(CSRC, "persistence.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    lines = r.stdout.strip().splitlines()
    assert lines[-1] == "ok", out[-4000:]
    built = int(lines[-2].split()[1].rstrip(","))
    assert built >= 80, lines[-2]
