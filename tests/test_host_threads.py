"""The host setup's row-parallel loops (sparse products, FSAI rows, adaptive
FSAI patterns, energy minimisation, power iterations, per-subsystem workers)
built with g++ under ThreadSanitizer and run on one setup with 1 and with 4
threads (MSP_SETUP_THREADS): no data race is reported, and the checksum of
every level's arrays and every subsystem's values is the same, i.e. the
result does not depend on the thread count.  Host code only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_05930_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_parallel_host_setup_is_race_free_and_thread_count_independent(tmp_path):
    exe = str(tmp_path / "check_host_setup_tsan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-ffp-contract=off", "-Wall", "-Wextra",
           "-Werror", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", os.path.join(CSRC, "host_setup.cpp"),
           os.path.join(ROOT, "tests", "native", "check_host_setup.cpp"), os.path.join(CSRC, "opts.cpp"),
           "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    sums = []
    for nt in ("1", "4"):
        env = dict(os.environ, MSP_SETUP_THREADS=nt, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
        r = subprocess.run([exe, "--checksum"], capture_output=True, text=True, env=env, timeout=900)
        assert r.returncode == 0, (nt, r.stdout[-2000:], r.stderr[-6000:])
        assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
        sums.append(r.stdout.strip().splitlines()[-1])
    assert sums[0].startswith("levels ") and sums[0] == sums[1], sums
