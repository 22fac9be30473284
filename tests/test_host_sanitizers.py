"""The library's host setup code (block extraction and validation, Alg. 2
coarsening, interpolation, FSAI, Galerkin products, per-subsystem values,
dense coarsest inverses) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer with every warning an error, and run on small
mirror-symmetric problems (tests/native/check_host_setup.cpp).  Host code
only: no GPU code is built with a sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_05930_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_host_setup_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "check_host_setup")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-Wall", "-Wextra", "-Werror",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", os.path.join(CSRC, "host_setup.cpp"),
           os.path.join(ROOT, "tests", "native", "check_host_setup.cpp"), os.path.join(CSRC, "opts.cpp"),
           "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host setup checks passed" in r.stdout
