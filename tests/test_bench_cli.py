"""bench.py's command line on the CPU: more than one GPU is refused with a
message and exit status 2 before anything touches a GPU (this solver has no
multi-GPU path), whether asked by --gpus or by a launcher's WORLD_SIZE."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ, **(env or {}))
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                          env=e, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    for args, env in ((["--gpus", "2"], None), (["--gpus", "8", "--steps", "3"], None), ([], {"WORLD_SIZE": "4"})):
        r = _run(args, env)
        assert r.returncode == 2, (args, r.returncode, r.stderr[-500:])
        assert "one GPU only" in r.stderr
        assert r.stdout == ""
