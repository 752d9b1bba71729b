"""The benchmark's command line on the host: its help text renders, and a
request for more than one GPU is refused with a message (the library has no
multi-GPU path)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_help_renders():
    r = _run("--help")
    assert r.returncode == 0, r.stderr
    assert "--gpus" in r.stdout and "--main-only" in r.stdout


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
